"""Dense displacement fields (T(x) = x + u(x)): value and dD/du per voxel
against the FP64 oracle, the chain rule back to an FFD, and SRWCRDenseLoss
against central differences of the oracle."""
import numpy as np
import pytest

from workloads import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def setup(S, w, role):
    fr, mr = torch.from_numpy(w.fixed).cuda(), torch.from_numpy(w.moving).cuda()
    flo, fhi = S.minmax(fr)
    mlo, mhi = S.minmax(mr)
    f = S.normalize(fr, flo, fhi, w.n_bins)
    m = S.normalize(mr, mlo, mhi, w.n_bins)
    prob = S.Problem(w.fixed_dims, w.moving_dims, w.n_bins, w.spatial_bins, w.ctrl_spacing, role)
    return f, m, prob, (flo, fhi, mlo, mhi)


def smooth_field(shape, sigma, k):
    from scipy import ndimage
    rng = np.random.default_rng(1804_05061 + 60 + k)
    u = rng.normal(0.0, 1.0, size=(3,) + tuple(shape))
    u = np.stack([ndimage.gaussian_filter(c, 3.0) for c in u])
    return (sigma * u / u.std()).astype(np.float32)


@pytest.mark.parametrize("role", [0, 1])
def test_dense_value_and_gradient_match_oracle(orc, role):
    import paper_1804_05061_amd as S
    w = synth.blobs(64)
    f, m, prob, r = setup(S, w, role)
    u = smooth_field(prob.field_shape[1:], 1.5, role)
    plan = S.Plan(prob)
    D, g = plan.grad_dense(f, m, torch.from_numpy(u).cuda())
    Dv = plan.eval_dense(f, m, torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    P = orc.Problem(w.fixed_dims, w.moving_dims, w.n_bins, w.spatial_bins, w.ctrl_spacing, role, dense=True)
    fo = orc.normalize(w.fixed, r[0], r[1], w.n_bins)
    mo = orc.normalize(w.moving, r[2], r[3], w.n_bins)
    Dr, gr = orc.gradient(P, fo, mo, u)
    gg = g.cpu().numpy().astype(np.float64)
    print(f"dense blobs64 role={role}: D={float(D):.12f} oracle={Dr:.12f} grad rel {rel(gg, gr):.2e}", flush=True)
    assert abs(float(D) - Dr) <= 1e-5 * Dr
    assert abs(float(Dv) - float(D)) <= 1e-12 * Dr
    assert rel(gg, gr) <= 1e-4


def test_dense_field_of_an_ffd_chains_to_the_ffd_gradient():
    """u sampled from an FFD on the GPU (ffd_warp of coordinate ramps) gives the
    FFD path's D, and sum_x beta_c(x) dD/du(x) gives its FFD gradient."""
    import paper_1804_05061_amd as S
    w = synth.blobs(48)
    f, m, prob, _ = setup(S, w, 0)
    ffd = synth.random_ffd(prob.ctrl_dims, 1.0, 3)
    plan = S.Plan(prob)
    D, g = plan.grad(f, m, torch.from_numpy(ffd).cuda())
    # u(x) = sum beta beta beta d, evaluated on the host in FP64 from the separable weights
    nx, ny, nz = prob.fixed_dims
    dl = prob.ctrl_spacing

    def axis_w(n, d):
        x = np.arange(n)
        p = x // d
        t = (x % d) / d
        B = np.stack([(1 - t) ** 3 / 6, (3 * t ** 3 - 6 * t ** 2 + 4) / 6, (-3 * t ** 3 + 3 * t ** 2 + 3 * t + 1) / 6,
                      t ** 3 / 6], axis=1)
        W = np.zeros((n, (n - 1) // d + 4))
        for l in range(4):
            W[x, p + l] = B[:, l]
        return W
    Wx, Wy, Wz = axis_w(nx, dl[0]), axis_w(ny, dl[1]), axis_w(nz, dl[2])
    u = np.einsum("zk,yj,xi,ekji->ezyx", Wz, Wy, Wx, ffd.astype(np.float64)).astype(np.float32)
    Dd, gd = plan.grad_dense(f, m, torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    gc = np.einsum("zk,yj,xi,ezyx->ekji", Wz, Wy, Wx, gd.cpu().numpy().astype(np.float64))
    print(f"dense vs ffd: D {float(Dd):.12f} vs {float(D):.12f}; chained grad rel {rel(gc, g.cpu().numpy()):.2e}",
          flush=True)
    assert abs(float(Dd) - float(D)) <= 1e-6 * float(D)
    assert rel(gc, g.cpu().numpy()) <= 1e-4


def test_dense_loss_backward_matches_finite_differences(orc):
    import paper_1804_05061_amd as S
    w = synth.blobs(40)
    f, m, prob, r = setup(S, w, 0)
    u = smooth_field(prob.field_shape[1:], 1.2, 5)
    plan = S.Plan(prob)
    uf = torch.from_numpy(u).cuda().requires_grad_(True)
    D = S.SRWCRDenseLoss.apply(uf, f, m, plan)
    (-1.5 * D).backward()
    g = uf.grad.detach().cpu().numpy().astype(np.float64) / -1.5
    P = orc.Problem(w.fixed_dims, w.moving_dims, w.n_bins, w.spatial_bins, w.ctrl_spacing, 0, dense=True)
    fo = orc.normalize(w.fixed, r[0], r[1], w.n_bins)
    mo = orc.normalize(w.moving, r[2], r[3], w.n_bins)
    rng = np.random.default_rng(1804_05061 + 61)
    # voxels with a clearly non-zero gradient, away from the grid edges
    Dr, gr = orc.gradient(P, fo, mo, u)
    cand = np.argwhere(np.abs(gr[:, 2:-2, 2:-2, 2:-2]) > 0.3 * np.abs(gr).max())
    pick = cand[rng.choice(len(cand), size=min(40, len(cand)), replace=False)]
    pts = [(int(e), int(z) + 2, int(y) + 2, int(x) + 2) for e, z, y, x in pick]
    fd = orc.fd_control_points(P, fo, mo, u, pts, 1e-3)
    ga = np.array([g[p] for p in pts])
    print(f"dense loss: vs FD {rel(ga, fd):.2e} (oracle analytic vs FD {rel(np.array([gr[p] for p in pts]), fd):.2e})",
          flush=True)
    assert rel(ga, fd) <= 1e-4                                 # oracle analytic vs FD: 1.5e-6
