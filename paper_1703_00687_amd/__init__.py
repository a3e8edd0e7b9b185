"""MI355X-native MSD radix sort of fixed-size records (RADULS2, arXiv 1703.00687).

The sorting itself runs in hand-written HIP kernels behind the C ABI declared
in ``include/raduls.h`` (``libraduls.so``, built from ``csrc/``).  The Python
modules here only marshal arguments (``binding``), generate synthetic inputs
(``workloads``), pick tuning parameters (``autotune``) and run a request loop
(``serve``).  The native library is loaded on first use and its absence is an
error: there is no fallback path.
"""
