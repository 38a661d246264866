"""Host sanitizer runs (no GPU): the FP64 oracle under AddressSanitizer and
UndefinedBehaviorSanitizer running its pins, and the library's host code under
AddressSanitizer running the CPU tests of its host logic (L-BFGS driver,
B-spline refinement, bending energy, argument checks).  Each run is a child
pytest process with the sanitizer runtime preloaded; any report fails it."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _pytest(files, env):
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", *files]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    return out


def test_oracle_pins_under_asan_and_ubsan():
    from oracle import oracle as O
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(libasan):
        pytest.skip("gcc's libasan not found")
    with tempfile.TemporaryDirectory() as tmp:
        lib = O.build(force=True, out=os.path.join(tmp, "liborc_san.so"), sanitize=True)
        env = dict(os.environ, ORC_LIB=lib, LD_PRELOAD=libasan, ASAN_OPTIONS="detect_leaks=0",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
        out = _pytest(["tests/test_oracle_pins.py"], env)
        print(out.strip().splitlines()[-1])


def test_host_library_under_asan():
    if subprocess.run(["which", "hipcc"], capture_output=True).returncode != 0:
        pytest.skip("hipcc not installed")
    from paper_1804_05061_amd import build as B
    rt = B.asan_runtime()
    if not rt:
        pytest.skip("clang ASan runtime not found")
    with tempfile.TemporaryDirectory() as tmp:
        lib = B.build_host_asan(os.path.join(tmp, "libsrwcr_asan.so"))
        env = dict(os.environ, SRWCR_LIB=lib, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0")
        out = _pytest(["tests/test_driver_cpu.py", "tests/test_abi.py"], env)
        print(out.strip().splitlines()[-1])
