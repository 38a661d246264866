"""register_lbfgs (Sec. II-F) end to end on a small CT-like pair: the cost
falls on every pyramid level and, at voxels next to tissue edges (where the
displacement is observable), the recovered displacement approaches the one
that generated the moving image."""
import numpy as np
import pytest

from workloads import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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
    # moving(x) = labels(x + u(x)): the registration should find T(x) ~ x - u(x)
    u, lab = w.meta["u"], w.meta["labels"]
    P = orc.Problem(w.fixed_dims, w.moving_dims, nb, (4, 4, 4), (8, 8, 8), 0)
    rng = np.random.default_rng(3)
    err0, err1 = [], []
    while len(err0) < 300:
        x, y, z = int(rng.integers(4, 60)), int(rng.integers(4, 60)), int(rng.integers(4, 44))
        blk = lab[z - 2:z + 3, y - 2:y + 3, x - 2:x + 3]
        if blk.min() == blk.max():
            continue
        d = orc.ffd_T(P, ffd, x, y, z) - np.array([x, y, z])
        target = -u[:, z, y, x]
        err0.append(np.sum(target ** 2))
        err1.append(np.sum((d - target) ** 2))
    rmse0, rmse1 = np.sqrt(np.mean(err0)), np.sqrt(np.mean(err1))
    print(f"{spatial}: edge displacement RMSE {rmse0:.3f} -> {rmse1:.3f} voxels", flush=True)
    assert rmse1 < 0.8 * rmse0
