"""Build guard (no GPU): the device code of the kernels, compiled with the
library's flags, holds no packed FP32 instruction (v_pk_{fma,mul,add}_f32),
and the same source compiled without the guard does -- so the check can fail."""
import os
import subprocess
import tempfile

import pytest

from paper_1804_05061_amd import build as B

pytestmark = pytest.mark.skipif(subprocess.run(["which", "hipcc"], capture_output=True).returncode != 0,
                                reason="hipcc not installed")


def test_kernels_hold_no_packed_fp32():
    asm = B.device_assembly("csrc/srwcr_kernels.hip")
    assert ".amdgcn_target" in asm and "gfx950" in asm
    found = [op for op in B.PACKED_FP32 if op in asm]
    assert not found, f"packed FP32 in the device code: {found}"


def test_guard_is_what_removes_them():
    """A float2 multiply-add that hipcc -O3 turns into v_pk_fma_f32 without the
    target feature, and into scalar FMAs with it."""
    src = ("#include <hip/hip_runtime.h>\n"
           "__global__ void k(float2 *a, const float2 *b, int n) { int i = blockIdx.x * blockDim.x + threadIdx.x;"
           " if (i < n) { float2 x = a[i], y = b[i]; a[i] = make_float2(x.x * y.x + 1.0f, x.y * y.y + 1.0f); } }\n")
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "k.hip")
        with open(path, "w") as fh:
            fh.write(src)
        outs = {}
        for name, flags in (("plain", [f for f in B.DEVICE_FLAGS if f not in ("-Xclang", "-target-feature",
                                                                              "-packed-fp32-ops")]),
                            ("guarded", B.DEVICE_FLAGS)):
            out = os.path.join(tmp, name + ".s")
            subprocess.run(["hipcc", "-O3", *flags, "-S", "-o", out, path], check=True, capture_output=True)
            outs[name] = open(out).read()
    assert any(op in outs["plain"] for op in B.PACKED_FP32)
    assert not any(op in outs["guarded"] for op in B.PACKED_FP32)
