"""register_lbfgs (Sec. II-F) end to end on a small synthetic pair: the cost
falls on every pyramid level and the recovered displacement approaches the
one that generated the moving image."""
import numpy as np
import pytest

from workloads import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_register_lbfgs_recovers_displacement(orc):
    import paper_1804_05061_amd as S
    w = synth.blobs(n=48)
    nb = 32
    f = S.normalize(torch.from_numpy(w.fixed).cuda(), float(w.fixed.min()), float(w.fixed.max()), nb)
    m = S.normalize(torch.from_numpy(w.moving).cuda(), float(w.moving.min()), float(w.moving.max()), nb)
    prob = S.Problem(w.fixed_dims, w.moving_dims, nb, (4, 4, 4), (6, 6, 6), S.MOVING_AS_A)
    ffd = np.zeros(prob.ffd_shape, dtype=np.float32)
    opts = S.LbfgsOptions(levels=2, max_iter=(40, 40, 0), stall_window=10, bending_weight=0.0)
    rep = S.register_lbfgs(prob, f, m, ffd, opts)
    print(rep, flush=True)
    for lvl in range(2):
        assert rep["final_value"][lvl] < rep["initial_value"][lvl]
        assert rep["iterations"][lvl] > 0
    # moving(x) = blobs(x + u(x)) * bias: the registration should find T(x) ~ x - u(x)
    u = w.meta["u"]                                          # (3, z, y, x) components x, y, z
    P = orc.Problem(w.fixed_dims, w.moving_dims, nb, (4, 4, 4), (6, 6, 6), 0)
    rng = np.random.default_rng(3)
    err0, err1 = [], []
    for _ in range(300):
        x, y, z = (int(v) for v in rng.integers(8, 40, size=3))
        d = orc.ffd_T(P, ffd, x, y, z) - np.array([x, y, z])
        target = -u[:, z, y, x]
        err0.append(np.sum(target ** 2))
        err1.append(np.sum((d - target) ** 2))
    rmse0, rmse1 = np.sqrt(np.mean(err0)), np.sqrt(np.mean(err1))
    print(f"displacement RMSE {rmse0:.3f} -> {rmse1:.3f} voxels", flush=True)
    assert rmse1 < 0.7 * rmse0
