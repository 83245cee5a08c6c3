"""The C-ABI validation paths under a host AddressSanitizer build of the library (CPU only):
invalid configurations, genotype and label values, scale grids and null handles are
rejected before any device work, with no out-of-bounds, use-after-free or double-free
access on the host side."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    c = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return c[-1] if c else None


def test_validation_paths_under_host_asan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("clang AddressSanitizer runtime not found")
    from paper_1106_0322_amd import build
    lib = build.ASAN_LIB
    if not os.path.exists(lib):
        build.build_asan()
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "asan_abi_driver.py"), lib], env=env,
                       capture_output=True, text=True, timeout=300)
    assert "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert "no sanitizer report" in r.stdout
