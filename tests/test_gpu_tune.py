"""Autotuning of a plan's launch shape: the tuned plan computes the same value
and gradient as the default plan (up to FP summation order) and the result
is cached per problem and device."""
import json

import numpy as np
import pytest

from workloads import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_tune_picks_a_shape_and_caches_it(tmp_path):
    import paper_1804_05061_amd as S
    w = synth.blobs(64)
    nb = 32
    P = S.Problem(w.fixed_dims, w.moving_dims, nb, w.spatial_bins, w.ctrl_spacing, S.MOVING_AS_A)
    f = S.normalize(torch.from_numpy(w.fixed).cuda(), float(w.fixed.min()), float(w.fixed.max()), nb)
    m = S.normalize(torch.from_numpy(w.moving).cuda(), float(w.moving.min()), float(w.moving.max()), nb)
    ffd = torch.from_numpy(synth.random_ffd(P.ctrl_dims, 1.0, 90)).cuda()
    cache = str(tmp_path / "tune.json")
    best = S.tune(P, f, m, ffd, steps=3, cache=cache)
    print("tuning", {k: v for k, v in best.items() if k != "timings"}, len(best["timings"]), flush=True)
    assert len(best["timings"]) >= 2 and best["ms"] == min(t["ms"] for t in best["timings"])
    assert S.tune(P, f, m, ffd, cache=cache) == json.load(open(cache))[next(iter(json.load(open(cache))))]
    D0, g0 = S.Plan(P).grad(f, m, ffd)
    for t in best["timings"]:
        D1, g1 = S.Plan(P, tuning=t).grad(f, m, ffd)
        torch.cuda.synchronize()
        assert abs(float(D1) - float(D0)) <= 1e-12 * float(D0)
        g0n, g1n = g0.cpu().numpy(), g1.cpu().numpy()
        assert np.linalg.norm(g1n - g0n) <= 1e-6 * np.linalg.norm(g0n)
    with pytest.raises(S.SrwcrError, match="INVALID_ARG"):
        S.Plan(P, tuning={"grad_item_voxels": -1})
