"""dD/ds_F, the derivative with respect to the normalised fixed volume, on
the GPU against the FP64 oracle (both roles, FFD and dense warps, and the
256x256x128 CT workload), and through the autograd Functions."""
import numpy as np
import pytest

from workloads import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def prepare(S, orc, w, role, dense, sigma, seed):
    P = S.Problem(w.fixed_dims, w.moving_dims, w.n_bins, w.spatial_bins, w.ctrl_spacing, role)
    flo, fhi, mlo, mhi = float(w.fixed.min()), float(w.fixed.max()), float(w.moving.min()), float(w.moving.max())
    f = S.normalize(torch.from_numpy(w.fixed).cuda(), flo, fhi, w.n_bins)
    m = S.normalize(torch.from_numpy(w.moving).cuda(), mlo, mhi, w.n_bins)
    if dense:
        rng = np.random.default_rng(1804_05061 + seed)
        disp = rng.normal(0.0, sigma, size=P.field_shape).astype(np.float32)
    else:
        disp = synth.random_ffd(P.ctrl_dims, sigma, seed)
    Po = orc.Problem(w.fixed_dims, w.moving_dims, w.n_bins, w.spatial_bins, w.ctrl_spacing, role, dense=dense)
    fo = orc.normalize(w.fixed, flo, fhi, w.n_bins)
    mo = orc.normalize(w.moving, mlo, mhi, w.n_bins)
    return P, f, m, disp, Po, fo, mo


@pytest.mark.parametrize("role", [0, 1])
@pytest.mark.parametrize("dense", [False, True])
def test_fixed_gradient_matches_oracle(orc, role, dense):
    import paper_1804_05061_amd as S
    w = synth.blobs(64)
    P, f, m, disp, Po, fo, mo = prepare(S, orc, w, role, dense, 1.0, 70 + role)
    plan = S.Plan(P)
    D, gF = plan.grad_fixed(f, m, torch.from_numpy(disp).cuda(), dense=dense)
    torch.cuda.synchronize()
    Dr, gr = orc.gradient_fixed(Po, fo, mo, disp)
    g = gF.cpu().numpy().astype(np.float64)
    print(f"dD/dF blobs64 role={role} dense={dense}: D rel {abs(float(D) - Dr) / Dr:.1e}, grad rel {rel(g, gr):.2e}",
          flush=True)
    assert abs(float(D) - Dr) <= 1e-5 * Dr
    assert rel(g, gr) <= 1e-4


def test_fixed_gradient_ct256_full_size(orc):
    import paper_1804_05061_amd as S
    w = synth.ct_phantom()
    P, f, m, disp, Po, fo, mo = prepare(S, orc, w, 0, False, 2.0, 2)
    plan = S.Plan(P)
    D, gF = plan.grad_fixed(f, m, torch.from_numpy(disp).cuda())
    torch.cuda.synchronize()
    Dr, gr = orc.gradient_fixed(Po, fo, mo, disp)
    g = gF.cpu().numpy().astype(np.float64)
    print(f"dD/dF ct256: D rel {abs(float(D) - Dr) / Dr:.1e}, grad rel {rel(g, gr):.2e}", flush=True)
    assert abs(float(D) - Dr) <= 1e-5 * Dr
    assert rel(g, gr) <= 1e-4


@pytest.mark.parametrize("dense", [False, True])
def test_autograd_fixed_input(orc, dense):
    """The loss Functions return dD/ds_F for a fixed volume that requires grad,
    scaled by grad_output, and the displacement gradient is unchanged."""
    import paper_1804_05061_amd as S
    w = synth.blobs(48)
    P, f, m, disp, Po, fo, mo = prepare(S, orc, w, 0, dense, 1.0, 72)
    plan = S.Plan(P)
    d = torch.from_numpy(disp).cuda().requires_grad_(True)
    fx = f.clone().requires_grad_(True)
    fn = S.SRWCRDenseLoss if dense else S.SRWCRLoss
    D = fn.apply(d, fx, m, plan)
    (3.0 * D).backward()
    torch.cuda.synchronize()
    _, gF = plan.grad_fixed(f, m, d.detach(), dense=dense)
    _, gd = plan.grad_dense(f, m, d.detach()) if dense else plan.grad(f, m, d.detach())
    torch.cuda.synchronize()
    assert rel(fx.grad.cpu().numpy(), 3.0 * gF.cpu().numpy()) <= 1e-6
    assert rel(d.grad.cpu().numpy(), 3.0 * gd.cpu().numpy()) <= 1e-6
    Dr, gr = orc.gradient_fixed(Po, fo, mo, disp)
    assert rel(fx.grad.cpu().numpy() / 3.0, gr) <= 1e-4
