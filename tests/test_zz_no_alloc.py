"""srwcr_grad_noalloc -- srwcr_grad on the library's static device workspace,
for callers that cannot allocate -- against srwcr_grad on a caller's
workspace, through the C ABI: two calls in a row, the second on a smaller
problem (the static array then holds the first call's contents), and the
rejection of a plan whose workspace exceeds the array."""
import ctypes

import numpy as np
import pytest

from workloads import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def case(S, n, crop, nb, seed):
    w = synth.blobs(n=n)
    nz, ny, nx = crop
    fixed = np.ascontiguousarray(w.fixed[:nz, :ny, :nx])
    moving = np.ascontiguousarray(w.moving[:nz, :ny, :nx])
    prob = S.Problem((nx, ny, nz), (nx, ny, nz), nb, (4, 4, 4), (6, 6, 6), S.MOVING_AS_A)
    f = S.normalize(torch.from_numpy(fixed).cuda(), float(fixed.min()), float(fixed.max()), nb)
    m = S.normalize(torch.from_numpy(moving).cuda(), float(moving.min()), float(moving.max()), nb)
    ffd = torch.from_numpy(synth.random_ffd(prob.ctrl_dims, 1.5, seed)).cuda()
    return prob, f, m, ffd


def noalloc_through_abi(S, plan, f, m, ffd):
    from paper_1804_05061_amd import _lib
    D = torch.full((), -1.0, dtype=torch.float64, device="cuda")
    g = torch.full(plan.problem.ffd_shape, np.nan, dtype=torch.float32, device="cuda")
    st = _lib.load().srwcr_grad_noalloc(plan.handle, f.data_ptr(), m.data_ptr(), ffd.data_ptr(), D.data_ptr(),
                                        g.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, _lib.load().srwcr_last_error().decode()
    torch.cuda.synchronize()
    return float(D.item()), g.cpu().numpy().astype(np.float64)


def test_noalloc_matches_workspace_calls_on_consecutive_problems():
    import paper_1804_05061_amd as S
    from paper_1804_05061_amd import _lib
    for n, crop, nb, seed in [(64, (64, 64, 64), 32, 41), (40, (30, 34, 40), 48, 42)]:
        prob, f, m, ffd = case(S, n, crop, nb, seed)
        plan = S.Plan(prob)
        assert plan.workspace_bytes <= _lib.NOALLOC_SCRATCH_BYTES
        D0, g0 = plan.grad(f, m, ffd)
        torch.cuda.synchronize()
        D0, g0 = float(D0.item()), g0.cpu().numpy().astype(np.float64)
        D1, g1 = noalloc_through_abi(S, plan, f, m, ffd)
        print(f"{crop} nb={nb}: workspace {plan.workspace_bytes} B; D {D1:.12f} vs {D0:.12f}, "
              f"gradient rel L2 {rel(g1, g0):.2e}", flush=True)
        # same kernels and partition, only the FP64 atomic order may differ
        assert abs(D1 - D0) <= 1e-12 * abs(D0)
        assert rel(g1, g0) <= 1e-6


def test_noalloc_rejects_a_plan_larger_than_the_static_workspace():
    import paper_1804_05061_amd as S
    from paper_1804_05061_amd import _lib
    prob = S.Problem((256, 256, 128), (256, 256, 128), 64, (6, 6, 6), (10, 10, 10), S.MOVING_AS_A)
    h = ctypes.c_void_p()
    assert _lib.load().srwcr_plan_create(ctypes.byref(prob.c()), ctypes.byref(h)) == 0
    try:
        assert _lib.load().srwcr_workspace_bytes(h) > _lib.NOALLOC_SCRATCH_BYTES
        st = _lib.load().srwcr_grad_noalloc(h, None, None, None, None, None, None)
        assert st == -3                                           # SRWCR_E_WORKSPACE
        assert b"static workspace" in _lib.load().srwcr_last_error()
    finally:
        _lib.load().srwcr_plan_destroy(h)
