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
    so u_xx = 2a everywhere and the energy is (2a)^2 at each of the control-node
    positions inside the grid: 9 x 5 x 4 nodes at spacing 5 in 41 x 21 x 16."""
    prob = S.Problem((41, 21, 16), (41, 21, 16), 32, (4, 4, 4), (5, 5, 5))
    ncx, ncy, ncz = prob.ctrl_dims
    a = 0.01
    ffd = np.zeros((3, ncz, ncy, ncx), dtype=np.float64)
    xi = (np.arange(ncx) - 1) * 5.0
    ffd[0] = (a * (xi ** 2 - 25.0 / 3.0))[None, None, :]
    E = bending(prob, ffd.astype(np.float32))
    npts = 9 * 5 * 4
    assert abs(E - 4 * a * a * npts) < 1e-6 * 4 * a * a * npts


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


def minimize(fg_py, x0, max_iter=500, history=5, stall_window=20, stall_tol=1e-12):
    """srwcr_lbfgs_minimize through the C ABI with a Python cost."""
    n = len(x0)
    x = np.ascontiguousarray(x0, dtype=np.float64).copy()

    def cb(user, xp, fp, gp):
        xx = np.ctypeslib.as_array(xp, shape=(n,))
        f, g = fg_py(xx.copy())
        fp[0] = f
        np.ctypeslib.as_array(gp, shape=(n,))[:] = g
        return 0

    c_cb = _lib.FG_FN(cb)
    it, ev, ff = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    st = _lib.load().srwcr_lbfgs_minimize(n, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), c_cb, None,
                                          max_iter, history, stall_window, stall_tol, ctypes.byref(it),
                                          ctypes.byref(ev), ctypes.byref(ff))
    return st, x, it.value, ev.value, ff.value


def test_lbfgs_minimizes_rosenbrock():
    """The optimiser of the registration driver (Sec. II-F: m = 5, backtracking
    Wolfe search) reaches the minimum (1, 1) of Rosenbrock's function."""
    def fg(x):
        a, b = x
        f = (1 - a) ** 2 + 100 * (b - a * a) ** 2
        g = np.array([-2 * (1 - a) - 400 * a * (b - a * a), 200 * (b - a * a)])
        return f, g
    st, x, it, ev, f = minimize(fg, [-1.2, 1.0])
    print(f"rosenbrock: status {st}, {it} iterations, {ev} evaluations, f={f:.3e}, x={x}")
    assert st == 0
    assert np.allclose(x, [1.0, 1.0], atol=1e-5) and f < 1e-10
    assert ev < 4 * it + 10


def test_lbfgs_ill_conditioned_quadratic():
    """A 60-dimensional quadratic with condition number 1e4: the minimiser is
    reached and every line search ends in an accepted step (no fallback)."""
    rng = np.random.default_rng(5)
    q, _ = np.linalg.qr(rng.normal(size=(60, 60)))
    A = q @ np.diag(np.logspace(0, 4, 60)) @ q.T
    b = rng.normal(size=60)
    xs = np.linalg.solve(A, b)

    def fg(x):
        r = A @ x - b
        return 0.5 * x @ A @ x - b @ x, r
    st, x, it, ev, f = minimize(fg, np.zeros(60), max_iter=2000)
    print(f"quadratic: status {st}, {it} iterations, {ev} evaluations")
    assert st == 0
    assert np.linalg.norm(x - xs) <= 1e-4 * np.linalg.norm(xs)


def test_lbfgs_line_search_terminates_on_a_kink():
    """|x| has no point where the curvature condition holds across the kink:
    the bracketed search shrinks its bracket instead of bouncing, and the run
    ends near 0 with the best point kept (status 0 or SRWCR_E_LINESEARCH)."""
    def fg(x):
        return float(np.abs(x).sum()), np.sign(x)
    st, x, it, ev, f = minimize(fg, [3.7, -2.2], max_iter=50, stall_window=5, stall_tol=1e-9)
    print(f"kink: status {st}, {it} iterations, {ev} evaluations, f={f:.3e}")
    assert st in (0, -7)
    assert f < 1e-2
    assert ev <= 41 * (it + 1) + 1


def test_lbfgs_callback_status_propagates():
    def fg(x):
        raise RuntimeError
    n = 3
    x = np.zeros(n)

    def cb(user, xp, fp, gp):
        return -6                                   # SRWCR_E_NONFINITE from the cost
    c_cb = _lib.FG_FN(cb)
    st = _lib.load().srwcr_lbfgs_minimize(n, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), c_cb, None, 10, 5,
                                          20, 1e-6, None, None, None)
    assert st == -6
