// Kernels for records of 64 bytes (every key width up to the record).
#include "raduls_kernels.hpp"

namespace raduls {
hipError_t run_rw8(const Params& P, uint32_t kw, hipStream_t s) { return run_rw<8>(P, kw, s); }
hipError_t serve_rw8(const Params& P, uint32_t kw, uint32_t wgs, hipStream_t s) {
  return serve_rw<8>(P, kw, wgs, s);
}
}  // namespace raduls
