"""Build libsrwcr.so in-tree for gfx950 with hipcc (no JIT, no torch extension).

Each HIP source is compiled in two steps: its device code alone, for gfx950,
with packed FP32 (v_pk_*_f32) turned off -- some of those instructions have
been seen to give wrong results on gfx950 -- then its host code alone,
embedding that device code object.  The target feature is a gfx950 one; kept
out of the host (x86) pass, it leaves the build log free of "not a
recognized feature" lines.  C++ sources are compiled as usual, and all
objects are linked into one shared library.  device_assembly() gives the
gfx950 assembly of a source as built here (a CPU test checks it for packed
FP32 instructions).
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/srwcr_kernels.hip", "csrc/srwcr_host.cpp", "csrc/srwcr_lbfgs.cpp", "csrc/srwcr_noalloc.hip"]
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc"),
          "-Wno-unused-command-line-argument"]
DEVICE_FLAGS = [
    "--offload-arch=" + ARCH, "--cuda-device-only",
    "-munsafe-fp-atomics",                       # native FP64 atomics in LDS and L2
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
HOST_FLAGS = ["--offload-arch=" + ARCH, "--cuda-host-only", "-munsafe-fp-atomics"]
PACKED_FP32 = ("v_pk_fma_f32", "v_pk_mul_f32", "v_pk_add_f32")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[:3]) + " ...")
    return r.stdout + r.stderr


def _object(src: str, tmp: str, verbose: bool, check: bool = False) -> str:
    path = os.path.join(HERE, src)
    stem = os.path.join(tmp, os.path.basename(src))
    obj = stem + ".o"
    extra = ["-DSRWCR_CHECK"] if check else []
    if src.endswith(".hip"):
        dev = stem + ".hipfb"
        _run(["hipcc", *COMMON, *extra, *DEVICE_FLAGS, "-c", "-o", dev, path], verbose)
        _run(["hipcc", *COMMON, *extra, *HOST_FLAGS, "-Xclang", "-fcuda-include-gpubinary", "-Xclang", dev, "-c",
              "-o", obj, path], verbose)
    else:
        _run(["hipcc", *COMMON, *extra, "-c", "-o", obj, path], verbose)
    return obj


def device_assembly(src: str = "csrc/srwcr_kernels.hip") -> str:
    """gfx950 assembly of one HIP source, compiled with the library's device flags."""
    with tempfile.TemporaryDirectory() as tmp:
        out = os.path.join(tmp, "k.s")
        _run(["hipcc", *COMMON, *DEVICE_FLAGS, "-S", "-o", out, os.path.join(HERE, src)], False)
        with open(out) as fh:
            return fh.read()


def build(verbose: bool = False, check: bool = False) -> str:
    """libsrwcr.so; check: the bounds-checked debug build (-DSRWCR_CHECK, see
    srwcr_debug_check_flags) as libsrwcr_check.so beside it."""
    out = os.path.join(HERE, "libsrwcr_check.so" if check else "libsrwcr.so")
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(len(SOURCES)) as ex:
            objs = list(ex.map(lambda s: _object(s, tmp, verbose, check), SOURCES))
        lib = os.path.join(tmp, "libsrwcr.so")
        _run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", lib, *objs], verbose)
        _copy(lib, out)
    return out


def build_host_asan(out: str, verbose: bool = False) -> str:
    """The library with its host code under AddressSanitizer (device code as
    in build()), into `out`, for CPU tests of the host logic; load it with the
    clang ASan runtime preloaded (asan_runtime())."""
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    with tempfile.TemporaryDirectory() as tmp:
        def obj(src):
            path = os.path.join(HERE, src)
            stem = os.path.join(tmp, os.path.basename(src))
            o = stem + ".o"
            if src.endswith(".hip"):
                dev = stem + ".hipfb"
                _run(["hipcc", *COMMON, *DEVICE_FLAGS, "-c", "-o", dev, path], verbose)
                _run(["hipcc", *COMMON, *HOST_FLAGS, *san, "-Xclang", "-fcuda-include-gpubinary", "-Xclang", dev,
                      "-c", "-o", o, path], verbose)
            else:
                _run(["hipcc", *COMMON, *san, "-c", "-o", o, path], verbose)
            return o
        with ThreadPoolExecutor(len(SOURCES)) as ex:
            objs = list(ex.map(obj, SOURCES))
        lib = os.path.join(tmp, "libsrwcr_asan.so")
        _run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", lib, *objs], verbose)
        _copy(lib, out)
    return out


def asan_runtime() -> str:
    """The clang AddressSanitizer runtime of this toolchain (for LD_PRELOAD)."""
    r = subprocess.run(["hipcc", "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        import glob
        found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
        path = found[-1] if found else ""
    return path


def _copy(src: str, dst: str) -> None:
    tmp = dst + ".tmp"
    with open(src, "rb") as fi, open(tmp, "wb") as fo:
        fo.write(fi.read())
    os.chmod(tmp, 0o755)
    os.replace(tmp, dst)


if __name__ == "__main__":
    print(build(verbose=True))
