"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/raduls.h declares, and rejects bad arguments before touching HIP."""

import os
import re

import pytest

from paper_1703_00687_amd import binding as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "raduls.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(raduls_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    syms = declared_symbols()
    for name in ("raduls_sort", "raduls_sort_batch", "raduls_tmp_bytes", "raduls_batch_ws_bytes",
                 "raduls_histogram", "raduls_partition", "raduls_strerror"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    lib = b.load()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert sorted(b.exported_symbols()) == declared_symbols()


def test_bad_record_and_key_sizes():
    for r in (0, 4, 12, 72, 128):
        assert b.raduls_sort(0, 0, 100, r, 8, raise_on_error=False) == b.E_UNSUPPORTED
    assert b.raduls_sort(0, 0, 100, 16, 0, raise_on_error=False) == b.E_INVALID
    assert b.raduls_sort(0, 0, 100, 16, 17, raise_on_error=False) == b.E_INVALID
    assert b.raduls_sort(0, 0, 1 << 32, 16, 8, raise_on_error=False) == b.E_UNSUPPORTED


def test_trivial_sizes_are_noops():
    for n in (0, 1):
        assert b.raduls_sort(0, 0, n, 16, 8, raise_on_error=False) == b.OK


def test_pointer_errors_rejected_on_host():
    assert b.raduls_sort(0, 4096, 100, 16, 8, raise_on_error=False) == b.E_INVALID
    assert b.raduls_sort(4096, 0, 100, 16, 8, raise_on_error=False) == b.E_INVALID
    assert b.raduls_sort(4096 + 8, 1 << 30, 100, 16, 8, raise_on_error=False) == b.E_ALIGN
    assert b.raduls_sort(4096, (1 << 30) + 4, 100, 16, 8, raise_on_error=False) == b.E_ALIGN
    # tmp overlapping recs
    assert b.raduls_sort(1 << 20, (1 << 20) + 256, 100, 16, 8, raise_on_error=False) == b.E_INVALID
    assert b.raduls_sort(1 << 20, (1 << 20) - 256, 100, 16, 8, raise_on_error=False) == b.E_INVALID


def test_step_argument_errors():
    ws = b.raduls_step_ws_bytes(1000, 16, 8)
    bad = [
        (16, 8, 0, 8),    # bits 0
        (16, 8, 65, 8),   # bits beyond the key
        (16, 8, 64, 0),   # width 0
        (16, 8, 64, 9),   # width > 8
    ]
    for r, k, bits, width in bad:
        st = b.raduls_histogram(1 << 20, 1000, r, k, bits, width, 1 << 21, 1 << 24, ws,
                                raise_on_error=False)
        assert st == b.E_INVALID
    st = b.raduls_histogram(1 << 20, 1000, 16, 8, 64, 8, 1 << 21, 1 << 24, ws - 1,
                            raise_on_error=False)
    assert st == b.E_TMP_SMALL
    st = b.raduls_partition(1 << 20, 1 << 20, 1000, 16, 8, 64, 8, 0, 1 << 24, ws,
                            raise_on_error=False)
    assert st == b.E_INVALID  # src == dst


def test_batch_argument_errors():
    ws = b.raduls_batch_ws_bytes(4, 1000, 16, 8)
    assert b.raduls_sort_batch(0, 0, 0, 16, 8, 0, 0, raise_on_error=False) == b.OK
    assert b.raduls_sort_batch(0, 4, 1000, 16, 8, 1 << 24, ws, raise_on_error=False) == b.E_INVALID
    assert b.raduls_sort_batch(1 << 20, 4, 1000, 16, 8, 1 << 24, ws - 1,
                               raise_on_error=False) == b.E_TMP_SMALL
    assert b.raduls_sort_batch(1 << 20, 4, 1000, 12, 8, 1 << 24, ws,
                               raise_on_error=False) == b.E_UNSUPPORTED


def test_size_queries():
    prev = 0
    for n in (2, 100, 10000, 1 << 20, 1 << 24, 1 << 28):
        t = b.raduls_tmp_bytes(n, 16, 8)
        assert t >= n * 16 and t >= prev
        prev = t
    # auxiliary workspace stays a small fraction of the data at scale
    assert b.raduls_tmp_bytes(1 << 28, 16, 8) < (1 << 28) * 16 * 1.10
    for r in range(8, 72, 8):
        for k in sorted({1, 8, min(16, r), r}):
            cap = b.raduls_mid_capacity(r, k)
            # the records and a 16-bit permutation of a job fit a CU's 160 KiB
            # of LDS
            assert cap >= 512 and cap % 64 == 0 and cap * (r + 2) <= 160 * 1024
    assert b.raduls_mid_capacity(12, 8) == 0
    assert b.raduls_mid_capacity(16, 17) == 0


def test_tuning_roundtrip_and_rejects():
    prev = b.raduls_set_tuning(digit_bits=5, tiny_max=64)
    try:
        t = b.raduls_get_tuning()
        assert t["digit_bits"] == 5 and t["tiny_max"] == 64
        with pytest.raises(b.RadulsError):
            b.raduls_set_tuning(digit_bits=9)
        with pytest.raises(b.RadulsError):
            b.raduls_set_tuning(tiny_max=1000)
    finally:
        b.raduls_set_tuning(**prev)
    assert b.raduls_get_tuning() == prev


def test_strerror():
    for st in (b.OK, b.E_INVALID, b.E_ALIGN, b.E_TMP_SMALL, b.E_UNSUPPORTED, b.E_HIP, b.E_DEVICE,
               b.E_SCRATCH, b.E_BUSY, b.E_STOPPED, b.E_TIMEOUT):
        assert b.strerror(st) and b.strerror(st) != "unknown status"


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes structs have the sizes and field offsets the C
    header gives (compiled here with the host compiler)."""
    import ctypes
    import shutil
    import subprocess
    from paper_1703_00687_amd import binding as b
    gcc = shutil.which("gcc")
    if gcc is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("no host compiler or HIP headers")
    src = tmp_path / "layout.c"
    src.write_text(
        "#include <stdio.h>\n#include <stddef.h>\n#include \"raduls.h\"\n"
        "int main(void) {\n"
        "  printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(raduls_tuning),\n"
        "         offsetof(raduls_tuning, lookback), offsetof(raduls_tuning, pair_hist),\n"
        "         offsetof(raduls_tuning, wave_job_max), offsetof(raduls_tuning, es_job_max),\n"
        "         sizeof(raduls_stats), offsetof(raduls_stats, moved_records),\n"
        "         offsetof(raduls_stats, pair_rounds), sizeof(raduls_array),\n"
        "         sizeof(raduls_bin), offsetof(raduls_bin, flags));\n"
        "  return 0;\n}\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.run([gcc, "-D__HIP_PLATFORM_AMD__", "-I", inc, "-I", "/opt/rocm/include", str(src),
                    "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                          text=True).stdout.split()]
    want = [ctypes.sizeof(b.raduls_tuning), b.raduls_tuning.lookback.offset,
            b.raduls_tuning.pair_hist.offset, b.raduls_tuning.wave_job_max.offset,
            b.raduls_tuning.es_job_max.offset, ctypes.sizeof(b.raduls_stats),
            b.raduls_stats.moved_records.offset, b.raduls_stats.pair_rounds.offset,
            ctypes.sizeof(b.raduls_array), ctypes.sizeof(b.raduls_bin), b.raduls_bin.flags.offset]
    assert got == want


def test_server_argument_errors_on_host():
    """Resident-server calls that fail before touching the device."""
    import ctypes
    lib = b.load()
    h = ctypes.c_void_p()
    assert lib.raduls_server_create(12, 8, 64, 1, 100, 0, ctypes.byref(h)) == b.E_UNSUPPORTED
    assert lib.raduls_server_create(16, 17, 64, 1, 100, 0, ctypes.byref(h)) == b.E_INVALID
    assert lib.raduls_server_create(16, 8, 0, 1, 100, 0, ctypes.byref(h)) == b.E_INVALID
    assert lib.raduls_server_create(16, 8, (1 << 20) + 1, 1, 100, 0, ctypes.byref(h)) == b.E_INVALID
    assert lib.raduls_server_create(16, 8, 64, 1, 600001, 0, ctypes.byref(h)) == b.E_INVALID
    assert lib.raduls_server_create(16, 8, 64, 1, 100, 600001, ctypes.byref(h)) == b.E_INVALID
    assert lib.raduls_server_create(16, 8, 64, 1, 100, 0, None) == b.E_INVALID
    t = ctypes.c_uint64()
    st = ctypes.c_uint32()
    assert lib.raduls_server_submit(None, None, 0, ctypes.byref(t)) == b.E_INVALID
    acc = ctypes.c_uint32()
    assert lib.raduls_server_submit_many(None, None, None, 0, ctypes.byref(t),
                                         ctypes.byref(acc)) == b.E_INVALID
    assert lib.raduls_server_poll(None, 0, ctypes.byref(st)) == b.E_INVALID
    assert lib.raduls_server_wait(None, 0, 1, ctypes.byref(st)) == b.E_INVALID
    assert lib.raduls_server_wait_range(None, 0, 1, 1, ctypes.byref(st)) == b.E_INVALID
    assert lib.raduls_server_info(None, None, None, None, None) == b.E_INVALID
    assert lib.raduls_server_completed(None, ctypes.byref(t), ctypes.byref(st)) == b.E_INVALID
    assert lib.raduls_server_destroy(None) == b.E_INVALID


def test_server_max_records_is_the_lds_capacity():
    for r, k in ((8, 8), (16, 8), (32, 16), (64, 64)):
        assert b.raduls_server_max_records(r, k) == b.raduls_mid_capacity(r, k)
    prev = b.raduls_set_tuning(mid_max=1000)
    try:
        assert b.raduls_server_max_records(16, 8) == 1000
    finally:
        b.raduls_set_tuning(**prev)
