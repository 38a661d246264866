"""The bounds-checked debug build (libsrwcr_check.so, SRWCR_CHECK) on the
parity workloads: no index check fails, and the results still match the FP64
oracle.  Runs in a child process that loads that build (SRWCR_LIB), one
process for all cases."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1804_05061_amd", "libsrwcr_check.so")

SCRIPT = r'''
import ctypes, sys
import numpy as np, torch
sys.path.insert(0, ROOT)
import paper_1804_05061_amd as S
from paper_1804_05061_amd import _lib
from oracle import oracle as O
from workloads import synth
L = _lib.load()
assert L._name == LIB, L._name
flags = ctypes.c_int32(0)
assert L.srwcr_debug_check_flags(ctypes.byref(flags), 1) == 0
def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
w = synth.blobs(n=48)
cases = [("blobs", w.fixed, w.moving, (4, 4, 4), (8, 8, 8)),
         ("ragged", w.fixed[:23, :29, :37], w.moving[:23, :29, :37], (5, 4, 6), (3, 4, 5)),
         ("nodes", w.fixed[:37, :43, :47], w.moving[:37, :43, :47], (0, 0, 0), (5, 4, 6)),
         ("unequal", w.fixed[:32, :36, :40], w.moving[:32:2, :36:2, :40:2], (5, 5, 5), (8, 8, 8))]
for name, fr, mr, K, d in cases:
    fr, mr = np.ascontiguousarray(fr), np.ascontiguousarray(mr)
    for role in (0, 1):
        nb = 32
        f = S.normalize(torch.from_numpy(fr).cuda(), float(fr.min()), float(fr.max()), nb)
        m = S.normalize(torch.from_numpy(mr).cuda(), float(mr.min()), float(mr.max()), nb)
        prob = S.Problem(fr.shape[::-1], mr.shape[::-1], nb, K, d, role)
        plan = S.Plan(prob)
        ffd = synth.random_ffd(prob.ctrl_dims, 1.0, 7)
        D, g = plan.grad(f, m, torch.from_numpy(ffd).cuda())
        Df, gF = plan.grad_fixed(f, m, torch.from_numpy(ffd).cuda())
        torch.cuda.synchronize()
        P = O.Problem(fr.shape[::-1], mr.shape[::-1], nb, K, d, role)
        fo, mo = f.cpu().numpy(), m.cpu().numpy()
        Dr, gr = O.gradient(P, fo, mo, ffd)
        ev, eg = abs(float(D) - Dr) / abs(Dr), rel(g.cpu().numpy().astype(np.float64), gr)
        assert L.srwcr_debug_check_flags(ctypes.byref(flags), 1) == 0
        print(f"{name} role {role}: value rel {ev:.1e} grad rel {eg:.1e} check flags {flags.value:#x}", flush=True)
        assert flags.value == 0 and ev < 1e-6 and eg < 1e-5
print("ok")
'''


def test_bounds_checked_build_records_no_violation():
    if not os.path.exists(LIB):
        pytest.skip("libsrwcr_check.so not built (__graft_entry__.build())")
    env = dict(os.environ, SRWCR_LIB=LIB)
    code = "ROOT = %r\nLIB = %r\n" % (ROOT, LIB) + SCRIPT
    r = subprocess.run([sys.executable, "-u", "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0 and r.stdout.strip().endswith("ok")
