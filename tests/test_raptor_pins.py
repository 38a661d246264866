"""Pins of the FP64 oracle's RaPTOR (eqs 6, 13, 14: boxcar patches, linear
window on A, frequency moments of B) against an independent numpy evaluation,
closed forms, an invariance and finite differences."""
import numpy as np
import pytest

from workloads import synth


def patches_for(shape_xyz, n, size, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape_xyz
    c = rng.integers(0, [nx, ny, nz], size=(n, 3))
    lo = c - size // 2
    return np.concatenate([lo, lo + size], axis=1).astype(np.int32)


def numpy_raptor(A, B, patches, nb):
    """Eqs (13), (14) written out in numpy: every bin, linear window h(t) = max(0, 1 - |t|)."""
    nz, ny, nx = A.shape
    tot = 0.0
    bins = np.arange(nb)
    for x0, y0, z0, x1, y1, z1 in patches:
        x0, y0, z0 = max(x0, 0), max(y0, 0), max(z0, 0)
        x1, y1, z1 = min(x1, nx), min(y1, ny), min(z1, nz)
        a = A[z0:z1, y0:y1, x0:x1].ravel().astype(np.float64)
        b = B[z0:z1, y0:y1, x0:x1].ravel().astype(np.float64)
        if a.size == 0:
            continue
        N = a.size
        H = np.maximum(0.0, 1.0 - np.abs(bins[None, :] - a[:, None]))        # [voxel, bin]
        p = H.sum(0) / N
        with np.errstate(invalid="ignore", divide="ignore"):
            mu = np.where(H.sum(0) > 0, (H * b[:, None]).sum(0) / H.sum(0), 0.0)
        var = (b * b).mean() - b.mean() ** 2
        if not var > 1e-5 * (b * b).mean():
            continue
        tot += ((b * b).mean() - (p * mu * mu).sum()) / var
    return tot / len(patches)


def problem(orc, dims, nb, role, d=4, dense=False):
    """dims = (nx, ny, nz); volumes are stored [nz][ny][nx]."""
    return orc.Problem(tuple(dims), tuple(dims), nb, (4, 4, 4), (d, d, d), role, dense=dense)


def pair(dims, k):
    return synth.smooth_pair(tuple(dims[::-1]), k=k)


@pytest.mark.parametrize("role", [0, 1])
def test_raptor_matches_numpy_definition(orc, role):
    fr, mr = pair((14, 13, 12), 7 + role)
    nb = 16
    f = orc.normalize(fr, fr.min(), fr.max(), nb)
    m = orc.normalize(mr, mr.min(), mr.max(), nb)
    P = problem(orc, (14, 13, 12), nb, role)
    ffd = synth.random_ffd(P.ctrl_dims, 0.8, 20 + role)
    pt = patches_for((14, 13, 12), 9, 6, 30 + role)
    v = orc.raptor(P, f, m, ffd, pt)
    w = orc.warp(P, m, ffd)
    A, B = (w, f.astype(np.float64)) if role == 0 else (f.astype(np.float64), w)
    ref = numpy_raptor(A, B, pt, nb)
    assert abs(v - ref) <= 1e-12 * max(1.0, abs(ref)), (v, ref)
    assert 0.0 <= v <= 1.0 + 1e-12


def test_raptor_zero_for_exact_function_on_bins(orc):
    """B = f(A), A on integer bins, one patch covering the grid: every mu_r(a)
    is f(a), so sum_a p mu^2 = E[B^2] and the patch term is 0."""
    rng = np.random.default_rng(41)
    nb = 12
    shape = (10, 9, 8)
    lab = rng.integers(0, nb, size=shape[::-1]).astype(np.float32)   # [nz][ny][nx]
    fmap = rng.uniform(0, nb - 1, size=nb).astype(np.float32)
    fixed = fmap[lab.astype(int)]                                     # B = f(A), role 0: moving is A
    P = problem(orc, shape, nb, 0)
    ffd = np.zeros((3,) + P.ctrl_dims[::-1], dtype=np.float32)
    pt = np.array([[0, 0, 0, 10, 9, 8]], dtype=np.int32)
    v = orc.raptor(P, fixed, lab, ffd, pt)
    assert abs(v) < 1e-12, v


def test_raptor_invariant_under_affine_B(orc):
    fr, mr = pair((12, 12, 10), 9)
    nb = 16
    f = orc.normalize(fr, fr.min(), fr.max(), nb)
    m = orc.normalize(mr, mr.min(), mr.max(), nb)
    P = problem(orc, (12, 12, 10), nb, 0)                            # fixed is B
    ffd = synth.random_ffd(P.ctrl_dims, 0.7, 22)
    pt = patches_for((12, 12, 10), 7, 6, 33)
    v0 = orc.raptor(P, f, m, ffd, pt)
    for a, b in [(0.5, 3.0), (-0.75, 12.0)]:
        v1 = orc.raptor(P, (a * f.astype(np.float64) + b).astype(np.float64).astype(np.float32), m, ffd, pt)
        assert abs(v1 - v0) <= 1e-6 * v0, (a, b, v0, v1)              # float32 storage of the rescaled B


@pytest.mark.parametrize("role", [0, 1])
@pytest.mark.parametrize("dense", [False, True])
def test_raptor_gradient_central_differences(orc, role, dense):
    fr, mr = pair((13, 12, 11), 11 + role)
    nb = 16
    f = orc.normalize(fr, fr.min(), fr.max(), nb)
    m = orc.normalize(mr, mr.min(), mr.max(), nb)
    P = problem(orc, (13, 12, 11), nb, role, dense=dense)
    rng = np.random.default_rng(50 + role)
    if dense:
        disp = rng.normal(0, 0.6, size=(3, 11, 12, 13)).astype(np.float32)
    else:
        disp = synth.random_ffd(P.ctrl_dims, 0.8, 24 + role)
    pt = patches_for((13, 12, 11), 10, 7, 35 + role)
    v, g = orc.raptor(P, f, m, disp, pt, want_grad=True)
    flat = np.argsort(-np.abs(g).ravel())[:30]
    h = 1e-4
    fd = []
    for i in flat:
        dp, dm_ = disp.copy().ravel(), disp.copy().ravel()
        dp[i] = np.float32(float(disp.ravel()[i]) + h)
        dm_[i] = np.float32(float(disp.ravel()[i]) - h)
        step = float(dp[i]) - float(dm_[i])
        fd.append((orc.raptor(P, f, m, dp.reshape(disp.shape), pt) - orc.raptor(P, f, m, dm_.reshape(disp.shape), pt)) / step)
    fd = np.array(fd)
    an = g.ravel()[flat]
    assert np.linalg.norm(fd - an) <= 1e-3 * np.linalg.norm(an), np.linalg.norm(fd - an) / np.linalg.norm(an)
