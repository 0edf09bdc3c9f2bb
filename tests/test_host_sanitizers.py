"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is rebuilt with both sanitizers on its host compilation (device
code unchanged), the sanitizer runtime is preloaded, and the C-ABI checks of
test_abi.py (loading, exports, struct layouts, the argument validation of
every entry point, handle creation without a device) run against that build
in a child process.  A heap or stack overrun, a use after free or undefined
behaviour on those paths stops the child with a report."""
import glob
import os
import subprocess
import sys

import pytest

from paper_2309_04623_amd import build as libbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return found[-1] if found else None


@pytest.mark.slow
def test_abi_checks_pass_under_host_sanitizers(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime in this toolchain")
    lib = libbuild.build(sanitize=True, out=str(tmp_path / "libnmf_san.so"))
    env = dict(os.environ, LD_PRELOAD=rt, NMF_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the child loads the sanitized build and runs with the sanitizer active
    probe = ("import ctypes; from paper_2309_04623_amd import nmf; nmf.lib(); "
             "ctypes.CDLL(None).__asan_init; print(nmf.LIB_PATH)")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0 and lib in r.stdout, r.stderr[-2000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_abi.py", "-q", "-p",
                        "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-3000:]
    assert r.returncode == 0, out[-3000:]
