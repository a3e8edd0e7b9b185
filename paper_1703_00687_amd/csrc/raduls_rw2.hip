// Kernels for records of 16 bytes (every key width up to the record).
#include "raduls_kernels.hpp"

namespace raduls {
hipError_t run_rw2(const Params& P, uint32_t kw, hipStream_t s) { return run_rw<2>(P, kw, s); }
}  // namespace raduls
