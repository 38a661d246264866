"""register_lbfgs (Sec. II-F) end to end on a small CT-like pair: the cost
falls on every pyramid level and, at voxels next to tissue edges (where the
displacement is observable), the recovered displacement approaches the one
that generated the moving image."""
import numpy as np
import pytest
from scipy import ndimage

from workloads import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def inverse_displacement(u, x, y, z, iters=60):
    """The warp T that undoes the generating field: moving(x) = labels(x + u(x))
    and fixed(x) = labels(x), so moving(T(x)) = fixed(x) needs
    T(x) + u(T(x)) = x.  Solved by the fixed-point iteration
    T <- x - u(T) (u trilinear between voxels), which contracts because
    |grad u| < 1 for these fields.  Returns T(x) - x.  For a field of 15 voxels
    the first-order answer -u(x) is off by |grad u| |u|, several voxels."""
    p = np.array([x, y, z], dtype=np.float64)
    t = p.copy()
    for _ in range(iters):
        coords = np.array([[t[2]], [t[1]], [t[0]]])          # (z, y, x) order of u[c]
        ut = np.array([ndimage.map_coordinates(u[c], coords, order=1, mode="nearest")[0] for c in range(3)])
        t = p - ut
    return t - p


def edge_rmse(orc, w, ffd, P, n=300, seed=3, margin=4):
    """RMSE over `n` random voxels next to tissue edges (where the displacement
    is observable) of T(x) - x against the inverse of the field that made the
    moving image (inverse_displacement)."""
    u, lab = w.meta["u"], w.meta["labels"]
    nz, ny, nx = lab.shape
    rng = np.random.default_rng(seed)
    err0, err1 = [], []
    while len(err0) < n:
        x = int(rng.integers(margin, nx - margin))
        y = int(rng.integers(margin, ny - margin))
        z = int(rng.integers(margin, nz - margin))
        blk = lab[z - 2:z + 3, y - 2:y + 3, x - 2:x + 3]
        if blk.min() == blk.max():
            continue
        d = orc.ffd_T(P, ffd, x, y, z) - np.array([x, y, z])
        target = inverse_displacement(u, x, y, z)
        err0.append(np.sum(target ** 2))
        err1.append(np.sum((d - target) ** 2))
    return float(np.sqrt(np.mean(err0))), float(np.sqrt(np.mean(err1)))


@pytest.mark.parametrize("spatial", [(4, 4, 4), (0, 0, 0)], ids=["K4", "nodes"])
def test_register_lbfgs_recovers_displacement(orc, spatial):
    """spatial (0, 0, 0): the regions sit on the FFD nodes at every level."""
    import paper_1804_05061_amd as S
    w = synth.ct_phantom(shape=(48, 64, 64), breathing=4.0, field_spacing=16, field_sigma=1.0, noise=20.0)
    nb = 32
    f = S.normalize(torch.from_numpy(w.fixed).cuda(), float(w.fixed.min()), float(w.fixed.max()), nb)
    m = S.normalize(torch.from_numpy(w.moving).cuda(), float(w.moving.min()), float(w.moving.max()), nb)
    prob = S.Problem(w.fixed_dims, w.moving_dims, nb, spatial, (8, 8, 8), S.MOVING_AS_A)
    ffd = np.zeros(prob.ffd_shape, dtype=np.float32)
    opts = S.LbfgsOptions(levels=2, max_iter=(40, 40, 0), stall_window=10, bending_weight=0.0)
    rep = S.register_lbfgs(prob, f, m, ffd, opts)
    print(rep, flush=True)
    for lvl in range(2):
        assert rep["final_value"][lvl] < rep["initial_value"][lvl]
        assert rep["iterations"][lvl] > 0
    # moving(x) = labels(x + u(x)): the registration should find T with T(x) + u(T(x)) = x
    P = orc.Problem(w.fixed_dims, w.moving_dims, nb, (4, 4, 4), (8, 8, 8), 0)
    rmse0, rmse1 = edge_rmse(orc, w, ffd, P)
    print(f"{spatial}: edge displacement RMSE {rmse0:.3f} -> {rmse1:.3f} voxels", flush=True)
    assert rmse1 < 0.8 * rmse0


@pytest.mark.timeout(900)
def test_register_ct256_three_levels_with_bending(orc):
    """Workload 2 registered as the paper does it (Sec. II-F, eq 1): the
    256x256x128 CT-like pair, 64 bins, 6x6x6 spatial bins, FFD spacing 10,
    three pyramid levels with at most 200 / 200 / 120 iterations, m = 5, a
    level stops when the cost is stable over 20 iterations, and the bending
    energy (summed over the control lattice) weighted by w_p = 0.1 (the
    mono-modal setting).  The cost falls on every level, no level ends in a
    failed line search, and the displacement error at tissue edges falls by
    at least 40 %.  (With C_p averaged over the lattice instead, w_p = 0.1
    leaves the FFD free to lower D to 0.02 -- below the 0.10 of the true
    field -- without recovering it: the edge error then grows.)"""
    import paper_1804_05061_amd as S
    w = synth.ct_phantom()
    nb = w.n_bins
    f = S.normalize(torch.from_numpy(w.fixed).cuda(), float(w.fixed.min()), float(w.fixed.max()), nb)
    m = S.normalize(torch.from_numpy(w.moving).cuda(), float(w.moving.min()), float(w.moving.max()), nb)
    prob = S.Problem(w.fixed_dims, w.moving_dims, nb, w.spatial_bins, w.ctrl_spacing, S.MOVING_AS_A)
    ffd = np.zeros(prob.ffd_shape, dtype=np.float32)
    opts = S.LbfgsOptions(levels=3, max_iter=(200, 200, 120), history=5, stall_window=20, bending_weight=0.1)
    rep = S.register_lbfgs(prob, f, m, ffd, opts)
    print(rep, flush=True)
    for lvl in range(3):
        assert rep["status"][lvl] == 0, rep
        assert rep["iterations"][lvl] > 0
        assert rep["final_value"][lvl] < rep["initial_value"][lvl]
    P = orc.Problem(w.fixed_dims, w.moving_dims, nb, w.spatial_bins, w.ctrl_spacing, 0)
    rmse0, rmse1 = edge_rmse(orc, w, ffd, P, n=400)
    print(f"ct256 3 levels, w_p 0.1: edge displacement RMSE {rmse0:.3f} -> {rmse1:.3f} voxels; seconds per level "
          f"{[round(t, 2) for t in rep['seconds']]}", flush=True)
    assert rmse1 < 0.6 * rmse0


def test_register_warm_start_reaches_the_coarsest_level(orc):
    """A caller's start is carried down the pyramid: starting a two-level run
    from the result of a first run gives the coarsest level a lower initial
    cost than starting from zero, and a different result."""
    import paper_1804_05061_amd as S
    w = synth.ct_phantom(shape=(48, 64, 64), breathing=4.0, field_spacing=16, field_sigma=1.0, noise=20.0)
    nb = 32
    f = S.normalize(torch.from_numpy(w.fixed).cuda(), float(w.fixed.min()), float(w.fixed.max()), nb)
    m = S.normalize(torch.from_numpy(w.moving).cuda(), float(w.moving.min()), float(w.moving.max()), nb)
    prob = S.Problem(w.fixed_dims, w.moving_dims, nb, (4, 4, 4), (8, 8, 8), S.MOVING_AS_A)
    opts = S.LbfgsOptions(levels=2, max_iter=(30, 30, 0), stall_window=10, bending_weight=0.0)
    ffd1 = np.zeros(prob.ffd_shape, dtype=np.float32)
    rep1 = S.register_lbfgs(prob, f, m, ffd1, opts)
    ffd2 = ffd1.copy()
    rep2 = S.register_lbfgs(prob, f, m, ffd2, opts)
    print(rep1["initial_value"], rep2["initial_value"], flush=True)
    assert rep2["initial_value"][0] < rep1["initial_value"][0]
    assert not np.array_equal(ffd2, ffd1)
    ffd3 = ffd1.copy()
    rep3 = S.register_lbfgs(prob, f, m, ffd3, S.LbfgsOptions(levels=1, max_iter=(0, 0, 0), stall_window=10))
    assert np.array_equal(ffd3, ffd1) and rep3["iterations"][0] == 0
