"""MI355X-native MSD radix sort of fixed-size records (RADULS2, arXiv 1703.00687).

The sorting itself runs in hand-written HIP kernels behind the C ABI declared
in ``include/raduls.h`` (``libraduls.so``, built from ``csrc/``).  The Python
modules here only marshal arguments (``binding``), generate synthetic inputs
(``workloads``), pick tuning parameters (``autotune``) and run a request loop
(``serve``).  The native library is loaded on first use and its absence is an
error: there is no fallback path.
"""

_BINDING_NAMES = {
    "sort", "sort_batch", "Batch", "RadulsError", "load",
    "raduls_tmp_bytes", "raduls_sort", "raduls_batch_ws_bytes", "raduls_sort_batch",
    "raduls_step_ws_bytes", "raduls_histogram", "raduls_partition", "raduls_check",
    "raduls_set_tuning", "raduls_get_tuning", "raduls_mid_capacity", "raduls_strerror",
    "raduls_set_profile_events",
}


def __getattr__(name):
    if name in _BINDING_NAMES:
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
