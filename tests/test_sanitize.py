"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle (every exported function, oracle/sanitize_main.cpp) and
the runtime's host side -- size queries, the workspace layout for many
shapes and tunings, the argument checks of every entry point
(tests/sanitize/runtime_host.hip, with the kernel launchers stubbed out and
the sanitizers applied to host code only)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", exe,
          os.path.join(ROOT, "oracle", "sanitize_main.cpp")])
    r = _run([exe], env=SAN_ENV)
    assert "ok" in r.stdout


HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("g++") is None,
                    reason="needs hipcc and g++")
def test_runtime_host_code_under_sanitizers(tmp_path):
    obj = str(tmp_path / "runtime_host.o")
    exe = str(tmp_path / "runtime_host")
    # device code is compiled as usual; the sanitizers instrument host code only
    _run([HIPCC, "-std=c++17", "-O1", "-g", "-fPIE", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-omit-frame-pointer",
          "-I", os.path.join(ROOT, "include"),
          "-I", os.path.join(ROOT, "paper_1703_00687_amd", "csrc"),
          "-c", os.path.join(ROOT, "tests", "sanitize", "runtime_host.hip"), "-o", obj])
    # the host link names no HIP source
    _run(["g++", "-fsanitize=address,undefined", obj, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = _run([exe], env=SAN_ENV)
    assert "ok" in r.stdout
