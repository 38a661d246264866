"""Host-side pieces of the registration driver (Sec. II-F), no GPU needed:
lattice refinement between pyramid levels and the bending-energy term of eq (1)."""
import ctypes

import numpy as np
import pytest

import paper_1804_05061_amd as S
from paper_1804_05061_amd import _lib
from workloads import synth


def refine(cnc, coarse, fnc):
    fine = np.zeros((3, fnc[2], fnc[1], fnc[0]), dtype=np.float32)
    c = (ctypes.c_int32 * 3)(*cnc)
    f = (ctypes.c_int32 * 3)(*fnc)
    _lib.check(_lib.load().srwcr_refine_ffd(c, coarse.ctypes.data_as(ctypes.c_void_p), f,
                                            fine.ctypes.data_as(ctypes.c_void_p)))
    return fine


def bending(prob, ffd, want_grad=False):
    g = np.zeros_like(ffd) if want_grad else None
    E = _lib.load().srwcr_bending_energy(ctypes.byref(prob.c()), ffd.ctypes.data_as(ctypes.c_void_p),
                                         g.ctypes.data_as(ctypes.c_void_p) if want_grad else None)
    return (E, g) if want_grad else E


@pytest.mark.parametrize("fdims,delta", [((40, 33, 26), (5, 4, 3)), ((64, 64, 32), (8, 8, 8))])
def test_refinement_reproduces_the_coarse_field(orc, fdims, delta):
    """u_f(2X) = 2 u_c(X): the refined lattice on the fine grid reproduces the
    doubled coarse displacement exactly (checked with the oracle's FFD)."""
    cdims = tuple((n + 1) // 2 for n in fdims)
    Pc = orc.Problem(cdims, cdims, 32, (4, 4, 4), delta, 0)
    Pf = orc.Problem(fdims, fdims, 32, (4, 4, 4), delta, 0)
    coarse = synth.random_ffd(Pc.ctrl_dims, 1.5, 21)
    fine = refine(Pc.ctrl_dims, coarse, Pf.ctrl_dims)
    rng = np.random.default_rng(0)
    for _ in range(40):
        X = [int(rng.integers(0, c)) for c in cdims]
        x = [2 * v for v in X]
        if any(a >= n for a, n in zip(x, fdims)):
            continue
        uc = orc.ffd_T(Pc, coarse, *X) - np.array(X)
        uf = orc.ffd_T(Pf, fine, *x) - np.array(x)
        assert np.allclose(uf, 2 * uc, atol=2e-5), (X, uf, 2 * uc)


def test_bending_energy_vanishes_on_affine_fields():
    prob = S.Problem((30, 26, 22), (30, 26, 22), 32, (4, 4, 4), (5, 4, 3))
    ncx, ncy, ncz = prob.ctrl_dims
    A = np.array([[0.02, -0.01, 0.03], [0.01, 0.0, -0.02], [-0.03, 0.02, 0.01]])
    ffd = np.zeros((3, ncz, ncy, ncx), dtype=np.float64)
    for k in range(ncz):
        for j in range(ncy):
            for i in range(ncx):
                ffd[:, k, j, i] = A @ np.array([(i - 1) * 5, (j - 1) * 4, (k - 1) * 3]) + 0.7
    assert abs(bending(prob, ffd.astype(np.float32))) < 1e-9


def test_bending_energy_of_a_quadratic_field():
    """u_x = a x^2 is reproduced by cubic B-spline coefficients a (x_i^2 - delta^2 / 3),
    so u_xx = 2a everywhere and the energy is (2a)^2."""
    prob = S.Problem((41, 21, 16), (41, 21, 16), 32, (4, 4, 4), (5, 5, 5))
    ncx, ncy, ncz = prob.ctrl_dims
    a = 0.01
    ffd = np.zeros((3, ncz, ncy, ncx), dtype=np.float64)
    xi = (np.arange(ncx) - 1) * 5.0
    ffd[0] = (a * (xi ** 2 - 25.0 / 3.0))[None, None, :]
    E = bending(prob, ffd.astype(np.float32))
    assert abs(E - 4 * a * a) < 1e-6 * 4 * a * a


def test_bending_energy_gradient_matches_differences():
    prob = S.Problem((24, 20, 18), (24, 20, 18), 32, (4, 4, 4), (4, 5, 6))
    ffd = synth.random_ffd(prob.ctrl_dims, 0.5, 22)
    E, g = bending(prob, ffd, want_grad=True)
    rng = np.random.default_rng(1)
    for idx in rng.choice(ffd.size, 30, replace=False):
        h = 1e-2
        p, m = ffd.copy().ravel(), ffd.copy().ravel()
        p[idx] += h
        m[idx] -= h
        fd = (bending(prob, p.reshape(ffd.shape)) - bending(prob, m.reshape(ffd.shape))) / (2 * h)
        assert abs(fd - g.ravel()[idx]) <= 1e-4 * max(1e-3, abs(fd)), (idx, fd, g.ravel()[idx])
