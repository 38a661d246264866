"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each one checks a closed
form, an invariant, a special case computed by an independent routine, brute
force on a tiny input, or finite differences.  Citations are to Gong et al.,
arXiv 1804.05061.
"""
import numpy as np
import pytest

from workloads import synth


def P(orc, nf, nb=32, K=(4, 4, 4), d=(5, 5, 5), role=0, nm=None):
    return orc.Problem(tuple(nf), tuple(nm or nf), nb, tuple(K), tuple(d), role)


def cubic_bspline_kernel(u):
    """Centred cubic B-spline B3(u) (independent closed form, not eq 8's pieces)."""
    u = abs(u)
    if u < 1:
        return 2.0 / 3.0 - u * u + 0.5 * u ** 3
    if u < 2:
        return (2 - u) ** 3 / 6.0
    return 0.0


# ------------------------------------------------------------------ eq (5)
def test_parzen_window_partition_and_continuity(orc):
    rng = np.random.default_rng(0)
    L = 31
    for s in np.concatenate([rng.uniform(0, L, 200), np.arange(0, L + 0.25, 0.5)]):
        tot = sum(orc.h(a - s) for a in range(L + 1))
        assert abs(tot - 1.0) < 1e-14, s
    assert orc.h(0.0) == 1.0
    for t0 in (0.5, 1.0):        # continuity at the piece joints
        assert abs(orc.h(t0 - 1e-12) - orc.h(t0 + 1e-12)) < 1e-10
    assert orc.h(1.0) == 0.0 and orc.h(1.5) == 0.0
    assert min(orc.h(t) for t in np.linspace(-1.2, 1.2, 1001)) >= 0.0


def test_parzen_one_sided_derivatives_match_differences(orc):
    eps = 1e-7
    for k in np.linspace(-1.4, 1.4, 57):
        left = (orc.h(k) - orc.h(k - eps)) / eps
        right = (orc.h(k + eps) - orc.h(k)) / eps
        assert abs(orc.dh(k, -1) - left) < 1e-5, k
        assert abs(orc.dh(k, +1) - right) < 1e-5, k
    # kinks at 0 and +-1: the two sides differ
    assert orc.dh(0.0, -1) == pytest.approx(0.1) and orc.dh(0.0, +1) == pytest.approx(-0.1)


# ------------------------------------------------------------------ eq (8)
def test_bspline_pieces_are_the_cubic_bspline(orc):
    for t in np.linspace(0, 1, 23):
        assert abs(sum(orc.beta(l, t) for l in range(4)) - 1.0) < 1e-15
        for l in range(4):
            assert abs(orc.beta(l, t) - cubic_bspline_kernel(t + 1 - l)) < 1e-15


def test_region_weights_partition_kernel_and_mirror(orc):
    for N, K in [(64, 4), (256, 6), (128, 6), (17, 5), (9, 8), (192, 5)]:
        spacing = (N - 1) / (K - 3)
        for x in range(N):
            w = orc.axis_region_weights(x, N, K)
            assert abs(w.sum() - 1.0) < 1e-14
            for j in range(K):                       # eq (7): B3 centred on node j at (j-1)*spacing
                assert abs(w[j] - cubic_bspline_kernel((x - (j - 1) * spacing) / spacing)) < 1e-12
            wm = orc.axis_region_weights(N - 1 - x, N, K)
            assert np.allclose(w, wm[::-1], atol=1e-13)


# ----------------------------------------------------------- eq (17), FFD
def test_ffd_constant_and_zero_displacement(orc):
    p = P(orc, (13, 11, 9), d=(4, 3, 5))
    ncx, ncy, ncz = p.ctrl_dims
    c = np.array([0.75, -1.25, 2.5], dtype=np.float32)
    ffd = np.broadcast_to(c[:, None, None, None], (3, ncz, ncy, ncx)).copy()
    for (x, y, z) in [(0, 0, 0), (12, 10, 8), (5, 7, 3), (3, 2, 4)]:
        T = orc.ffd_T(p, ffd, x, y, z)
        assert np.allclose(T, np.array([x, y, z]) + c, atol=1e-13)
        T0 = orc.ffd_T(p, np.zeros_like(ffd), x, y, z)
        assert np.array_equal(T0, [x, y, z])


def test_ffd_linear_precision(orc):
    """Cubic B-splines reproduce linear functions: coefficients sampled from an
    affine map at node positions (paper index i at i*delta) give that map."""
    p = P(orc, (21, 17, 13), d=(5, 4, 3))
    ncx, ncy, ncz = p.ctrl_dims
    Amat = np.array([[0.01, -0.02, 0.03], [0.0, 0.015, -0.01], [-0.02, 0.005, 0.01]])
    ffd = np.zeros((3, ncz, ncy, ncx), dtype=np.float64)
    for k in range(ncz):
        for j in range(ncy):
            for i in range(ncx):
                pos = np.array([(i - 1) * 5, (j - 1) * 4, (k - 1) * 3], dtype=np.float64)
                ffd[:, k, j, i] = Amat @ pos
    ffd = ffd.astype(np.float32)
    for (x, y, z) in [(0, 0, 0), (20, 16, 12), (7, 9, 5), (13, 3, 11)]:
        T = orc.ffd_T(p, ffd, x, y, z)
        exp = np.array([x, y, z]) + Amat @ np.array([x, y, z])
        assert np.allclose(T, exp, atol=2e-6)        # float32 coefficients


def test_integer_shift_warp_is_a_shift(orc):
    rng = np.random.default_rng(1)
    nx, ny, nz = 12, 10, 8
    mov = rng.uniform(0, 31, size=(nz, ny, nx)).astype(np.float32)
    p = P(orc, (nx, ny, nz), d=(3, 3, 3))
    ncx, ncy, ncz = p.ctrl_dims
    ffd = np.zeros((3, ncz, ncy, ncx), dtype=np.float32)
    ffd[0] += 2.0
    ffd[1] -= 1.0
    w = orc.warp(p, mov, ffd)
    assert np.allclose(w[:, 1:, :nx - 2], mov[:, :ny - 1, 2:], atol=1e-12)
    w0 = orc.warp(p, mov, np.zeros_like(ffd))
    assert np.array_equal(w0, mov.astype(np.float64))


# ------------------------------------------------------- trilinear sample
def test_trilinear_reproduces_affine_and_gradient(orc):
    nx, ny, nz = 7, 6, 5
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    vol = (1.5 + 0.25 * x - 0.5 * y + 0.125 * z).astype(np.float32)
    p = P(orc, (nx, ny, nz))
    rng = np.random.default_rng(2)
    for _ in range(50):
        yy = rng.uniform([0, 0, 0], [nx - 1, ny - 1, nz - 1])
        v, g = orc.sample(p, vol, yy)
        assert abs(v - (1.5 + 0.25 * yy[0] - 0.5 * yy[1] + 0.125 * yy[2])) < 1e-12
        assert np.allclose(g, [0.25, -0.5, 0.125], atol=1e-12)
    v, g = orc.sample(p, vol, [-3.0, 2.5, 10.0])     # clamped x and z
    assert abs(v - (1.5 + 0 - 1.25 + 0.5)) < 1e-12
    assert g[0] == 0.0 and g[2] == 0.0 and abs(g[1] + 0.5) < 1e-12


# ------------------------------------------- unequal fixed / moving grids
@pytest.mark.parametrize("nf,nm", [((16, 12, 10), (8, 6, 5)), ((8, 9, 10), (12, 9, 15))])
def test_unequal_grid_mapping_closed_form(orc, nf, nm):
    """Voxel centres of the two grids coincide in physical space: fixed voxel x
    maps to moving coordinate y = (T(x) + 1/2) M / N - 1/2 per axis, clamped to
    [0, M - 1] (the interpolation reading of Sec. II-F).  A moving image that
    is affine in its own index coordinates is reproduced exactly at every
    fixed voxel, for a constant displacement c (T = x + c) on both a coarser
    and a finer moving grid; the x axis here takes both signs of c."""
    mz, my, mx = np.meshgrid(np.arange(nm[2]), np.arange(nm[1]), np.arange(nm[0]), indexing="ij")
    ramp = lambda a, b, c: 9.0 + 0.75 * a - 0.5 * b + 0.25 * c      # stays inside [0, 31]
    mov = ramp(mx, my, mz).astype(np.float32)
    for shift in ((0.0, 0.0, 0.0), (1.25, -0.5, 0.75), (-2.0, 1.5, 0.0)):
        p = P(orc, nf, nb=32, K=(4, 4, 4), d=(3, 3, 3), nm=nm)
        ncx, ncy, ncz = p.ctrl_dims
        ffd = np.zeros((3, ncz, ncy, ncx), dtype=np.float32)
        for e in range(3):
            ffd[e] = shift[e]
        got = orc.warp(p, mov, ffd)
        z, y, x = np.meshgrid(np.arange(nf[2]), np.arange(nf[1]), np.arange(nf[0]), indexing="ij")
        yy = []
        for e, xe in enumerate((x, y, z)):
            ye = (xe + shift[e] + 0.5) * nm[e] / nf[e] - 0.5
            yy.append(np.clip(ye, 0.0, nm[e] - 1))
        exp = ramp(*yy)
        assert np.abs(got - exp).max() < 1e-12, (nf, nm, shift, np.abs(got - exp).max())


@pytest.mark.parametrize("role", [0, 1])
def test_unequal_grid_gradient_central_differences(orc, role):
    """The chain factor dy/dT = M / N of the grid mapping (eq 16): a 16^3 fixed
    and an 8^3 moving volume (every second voxel of a smooth pair), delta 5,
    K = 4, 32 bins, Phi ~ N(0, 1 vox).  The analytic gradient agrees with
    central differences of full re-evaluations; without the factor 1/2 it
    would be off by a factor 2 on every component."""
    fr, mr = synth.smooth_pair((16, 16, 16), k=3 + role)
    mr = np.ascontiguousarray(mr[::2, ::2, ::2])
    nb = 32
    f = orc.normalize(fr, fr.min(), fr.max(), nb)
    m = orc.normalize(mr, mr.min(), mr.max(), nb)
    p = P(orc, (16, 16, 16), nb=nb, K=(4, 4, 4), d=(5, 5, 5), role=role, nm=(8, 8, 8))
    ffd = synth.random_ffd(p.ctrl_dims, 1.0, 30 + role)
    D, g = orc.gradient(p, f, m, ffd)
    flat = np.argsort(-np.abs(g).ravel())
    idx = flat[:60]
    hstep = 1e-4
    fd = []
    for i in idx:
        e = np.zeros(g.size, dtype=np.float64)
        e[i] = hstep
        fp_ = (ffd.astype(np.float64).ravel() + e).astype(np.float32)
        fm_ = (ffd.astype(np.float64).ravel() - e).astype(np.float32)
        hh = (fp_.astype(np.float64) - fm_.astype(np.float64))[i]
        fd.append((orc.value(p, f, m, fp_.reshape(ffd.shape)) - orc.value(p, f, m, fm_.reshape(ffd.shape))) / hh)
    fd = np.array(fd)
    an = g.ravel()[idx]
    rel = np.linalg.norm(fd - an) / np.linalg.norm(an)
    print(f"unequal grids role={role}: D={D:.6f} FD rel {rel:.2e}")
    assert rel < 1e-3, rel


# ----------------------------------------------------- normalisation
def test_normalize_is_ieee_single_formula(orc):
    rng = np.random.default_rng(3)
    raw = rng.normal(0, 300, size=10000).astype(np.float32)
    lo, hi = float(raw.min()), float(raw.max())
    out = orc.normalize(raw, lo, hi, 64)
    exp = (raw - np.float32(lo)) * np.float32(63.0 / (hi - lo))    # numpy float32 ops round per op
    exp = np.clip(exp, 0, 63).astype(np.float32)
    assert np.array_equal(out, exp)
    assert out.min() == 0.0 and abs(out.max() - 63.0) < 1e-4


# ---------------------------------------------------------- eqs (3), (4)
def test_joint_pdf_sums_and_region_marginal(orc):
    w1 = synth.blobs(n=16)
    p = P(orc, (16, 16, 16), K=(4, 5, 4))
    f = orc.normalize(w1.fixed, w1.fixed.min(), w1.fixed.max(), 32)
    m = orc.normalize(w1.moving, w1.moving.min(), w1.moving.max(), 32)
    ffd = synth.random_ffd(p.ctrl_dims, 0.7, 1)
    pdf, Z = orc.joint_pdf(p, f, m, ffd)
    assert abs(pdf.sum() - 1.0) < 1e-13
    assert abs(Z - 16 ** 3) < 1e-9                       # sum_r w = 1 at every voxel
    # p(r) = (1/Z) sum_x w(r, x): independent of the images
    pdf2, _ = orc.joint_pdf(p, m, f, np.zeros_like(ffd))
    pr_exp = np.zeros(p.n_regions)
    for z in range(16):
        wz = orc.axis_region_weights(z, 16, 4)
        for y in range(16):
            wy = orc.axis_region_weights(y, 16, 5)
            for x in range(16):
                wx = orc.axis_region_weights(x, 16, 4)
                pr_exp += np.einsum("k,j,i->kji", wz, wy, wx).ravel()
    pr_exp /= 16 ** 3
    assert np.allclose(pdf.sum(axis=(1, 2)), pr_exp, atol=1e-14)
    assert np.allclose(pdf2.sum(axis=(1, 2)), pr_exp, atol=1e-14)


def test_joint_pdf_brute_force_all_bins(orc):
    """Literal eq (3) over every (a, b, r) on a tiny volume vs the oracle's tap-restricted sum."""
    rng = np.random.default_rng(4)
    nx, ny, nz, nb = 5, 4, 4, 8
    p = P(orc, (nx, ny, nz), nb=nb, K=(4, 4, 5), d=(2, 2, 2), role=1)
    f = rng.uniform(0, nb - 1, size=(nz, ny, nx)).astype(np.float32)
    f[0, 0, 0], f[1, 1, 1] = 0.0, nb - 1.0                 # range ends
    m = rng.uniform(0, nb - 1, size=(nz, ny, nx)).astype(np.float32)
    ffd = synth.random_ffd(p.ctrl_dims, 0.6, 4)
    pdf, Z = orc.joint_pdf(p, f, m, ffd)
    warped = orc.warp(p, m, ffd)
    ref = np.zeros_like(pdf)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                w = np.einsum("k,j,i->kji", orc.axis_region_weights(z, nz, 5), orc.axis_region_weights(y, ny, 4),
                              orc.axis_region_weights(x, nx, 4)).ravel()
                A, B = float(f[z, y, x]), warped[z, y, x]        # role 1: moving is B
                ha = np.array([orc.h(a - A) for a in range(nb)])
                hb = np.array([orc.h(b - B) for b in range(nb)])
                ref += w[:, None, None] * ha[None, :, None] * hb[None, None, :]
    assert abs(ref.sum() - Z) < 1e-10
    assert np.allclose(pdf, ref / ref.sum(), atol=1e-15)


def test_joint_mass_boxes_partition_the_pdf(orc):
    """Eq (3) is a sum over voxels: the box masses of a partition of the grid add
    up to Z p, and each box holds exactly its voxel count (sum_r w = 1 and the
    Parzen window sums to 1 in both images)."""
    w1 = synth.blobs(n=16)
    p = P(orc, (16, 14, 12), K=(4, 5, 4), nb=16, role=1)
    f = orc.normalize(w1.fixed[:12, :14, :16], w1.fixed.min(), w1.fixed.max(), 16)
    m = orc.normalize(w1.moving[:12, :14, :16], w1.moving.min(), w1.moving.max(), 16)
    ffd = synth.random_ffd(p.ctrl_dims, 0.8, 2)
    pdf, Z = orc.joint_pdf(p, f, m, ffd)
    q = np.zeros_like(pdf)
    for xs in ((0, 7), (7, 16)):
        for ys in ((0, 3), (3, 14)):
            for zs in ((0, 5), (5, 9), (9, 12)):
                box = xs + ys + zs
                qb = orc.joint_mass_box(p, f, m, ffd, box)
                nvox = (xs[1] - xs[0]) * (ys[1] - ys[0]) * (zs[1] - zs[0])
                assert abs(qb.sum() - nvox) < 1e-10 * nvox
                q += qb
    assert np.allclose(q, pdf * Z, rtol=0, atol=1e-12)


def test_fd_harness_matches_full_reevaluation(orc):
    """The support-box finite differences equal central differences of full
    re-evaluations of D (perturbing one node changes T only where the node's
    cubic B-spline weight can be non-zero, eq 17)."""
    fr, mr = synth.smooth_pair((18, 16, 15), k=3)
    p = P(orc, (18, 16, 15), nb=24, K=(4, 4, 5), d=(4, 5, 4), role=0)
    f = orc.normalize(fr, fr.min(), fr.max(), 24)
    m = orc.normalize(mr, mr.min(), mr.max(), 24)
    ffd = synth.random_ffd(p.ctrl_dims, 1.0, 5)
    pts = [(0, 2, 3, 2), (1, 4, 2, 5), (2, 3, 4, 3), (0, 0, 0, 0), (2, 6, 6, 7)]
    h = 1e-3
    fd = orc.fd_control_points(p, f, m, ffd, pts, h)
    for (e, k, j, i), v in zip(pts, fd):
        fp_, fm_ = ffd.copy(), ffd.copy()
        fp_[e, k, j, i] = np.float32(float(ffd[e, k, j, i]) + h)
        fm_[e, k, j, i] = np.float32(float(ffd[e, k, j, i]) - h)
        ref = (orc.value(p, f, m, fp_) - orc.value(p, f, m, fm_)) / (float(fp_[e, k, j, i]) - float(fm_[e, k, j, i]))
        assert abs(v - ref) <= 1e-12 + 1e-7 * abs(ref), (e, k, j, i, v, ref)   # D rounding / 2h ~ 1e-14


# ------------------------------------------------- eqs (9), (11), (12)
@pytest.mark.parametrize("role", [0, 1])
def test_srwcr_forms_agree_and_range(orc, role):
    w1 = synth.blobs(n=20)
    p = P(orc, (20, 20, 20), K=(4, 4, 5), role=role)
    f = orc.normalize(w1.fixed, w1.fixed.min(), w1.fixed.max(), 32)
    m = orc.normalize(w1.moving, w1.moving.min(), w1.moving.max(), 32)
    ffd = synth.random_ffd(p.ctrl_dims, 1.0, 2)
    pdf, Z = orc.joint_pdf(p, f, m, ffd)
    vals = [orc.srwcr_from_pdf(pdf, w) for w in range(4)]
    assert max(vals) - min(vals) < 1e-13
    assert 0.0 <= vals[0] <= 1.0
    assert abs(orc.value(p, f, m, ffd) - vals[0]) < 1e-15


# ------------------------------------- exact functional dependence: D = 0
@pytest.mark.parametrize("role", [0, 1])
def test_D_zero_for_exact_function_on_bin_centres(orc, role):
    """B = f(A) with both images integer-valued (bin centres): every regional
    conditional variance is zero, so D = 0 and 1 - D = 1 (Sec. II-D)."""
    rng = np.random.default_rng(5)
    nx, ny, nz, nb = 12, 11, 10, 16
    labels = rng.integers(0, nb, size=(nz, ny, nx))
    fmap = rng.permutation(nb)                               # injective, non-monotone
    A = labels.astype(np.float32)
    B = fmap[labels].astype(np.float32)
    p = P(orc, (nx, ny, nz), nb=nb, K=(4, 4, 4), d=(3, 3, 3), role=role)
    fixed, moving = (B, A) if role == 0 else (A, B)
    ffd = np.zeros((3,) + p.ctrl_dims[::-1], dtype=np.float32)
    D = orc.value(p, fixed, moving, ffd)
    assert abs(D) < 1e-14
    # a non-functional pair is strictly positive
    D2 = orc.value(p, fixed, rng.permutation(moving.ravel()).reshape(moving.shape), ffd)
    assert D2 > 1e-3


# ---------------------------------- one constant region: D = 1 - CR, eq (2)
def global_cr_numpy(A, B, nb):
    """Correlation ratio of eq (2) from a 2-D Parzen histogram (independent numpy)."""
    def weights(s):
        s = s.ravel().astype(np.float64)
        k = np.minimum(np.floor(s), nb - 2).astype(int)
        t = s - k
        w0 = np.where(t < 0.5, 1 - 0.1 * t - 1.8 * t * t, 1.9 - 3.7 * t + 1.8 * t * t)
        Wm = np.zeros((s.size, nb))
        Wm[np.arange(s.size), k] += w0
        Wm[np.arange(s.size), k + 1] += 1 - w0
        return Wm
    H = weights(A).T @ weights(B)                       # (a, b)
    H /= H.sum()
    pa, pb = H.sum(1), H.sum(0)
    b = np.arange(nb)
    mu = (b * pb).sum()
    var = (b * b * pb).sum() - mu * mu
    nz = pa > 0
    mua = (H[nz] @ b) / pa[nz]
    vara = (H[nz] @ (b * b)) / pa[nz] - mua ** 2
    return 1.0 - (vara * pa[nz]).sum() / var


@pytest.mark.parametrize("role", [0, 1])
def test_single_region_is_global_correlation_ratio(orc, role):
    w1 = synth.blobs(n=18)
    nb = 32
    f = orc.normalize(w1.fixed, w1.fixed.min(), w1.fixed.max(), nb)
    m = orc.normalize(w1.moving, w1.moving.min(), w1.moving.max(), nb)
    p = P(orc, (18, 18, 18), nb=nb, K=(1, 1, 1), role=role)
    ffd = synth.random_ffd(p.ctrl_dims, 1.0, 3)
    D = orc.value(p, f, m, ffd)
    warped = orc.warp(p, m, ffd)
    A, B = (warped, f) if role == 0 else (f, warped)
    assert abs(D - (1.0 - global_cr_numpy(A, B, nb))) < 1e-13


# -------------------------------------------- affine rescaling invariance
@pytest.mark.parametrize("role", [0, 1])
def test_affine_rescaling_of_moving_leaves_D_unchanged(orc, role):
    """An increasing affine map is removed exactly by the min-max normalisation;
    a decreasing one flips s -> L - s, an exact symmetry of both roles."""
    w1 = synth.blobs(n=16)
    nb = 32
    raw_m = np.rint(31 * (w1.moving - w1.moving.min()) / (w1.moving.max() - w1.moving.min())).astype(np.float32)
    f = orc.normalize(w1.fixed, w1.fixed.min(), w1.fixed.max(), nb)
    p = P(orc, (16, 16, 16), nb=nb, K=(4, 4, 4), role=role)
    ffd = synth.random_ffd(p.ctrl_dims, 1.0, 5)
    D0 = orc.value(p, f, orc.normalize(raw_m, 0, 31, nb), ffd)
    up = (2 * raw_m + 5).astype(np.float32)               # exact in float32
    D1 = orc.value(p, f, orc.normalize(up, 5, 67, nb), ffd)
    down = (31 - raw_m).astype(np.float32)
    D2 = orc.value(p, f, orc.normalize(down, 0, 31, nb), ffd)
    assert abs(D1 - D0) < 1e-14
    assert abs(D2 - D0) < 1e-13
    # a non-linear monotone map is not an exact symmetry (bins are linear in intensity)
    sq = (raw_m ** 2).astype(np.float32)
    D3 = orc.value(p, f, orc.normalize(sq, 0, 961, nb), ffd)
    assert abs(D3 - D0) > 1e-6


# ------------------------------------------------------ gradient algebra
@pytest.mark.parametrize("role", [0, 1])
def test_gradient_eq19_21_match_eq18_20(orc, role):
    w1 = synth.blobs(n=14)
    nb = 16
    f = orc.normalize(w1.fixed, w1.fixed.min(), w1.fixed.max(), nb)
    m = orc.normalize(w1.moving, w1.moving.min(), w1.moving.max(), nb)
    p = P(orc, (14, 14, 14), nb=nb, K=(4, 5, 4), d=(4, 4, 4), role=role)
    ffd = synth.random_ffd(p.ctrl_dims, 0.8, 6)
    D0, g0, dm0 = orc.gradient(p, f, m, ffd, form=0, want_dDdM=True)
    D1, g1, dm1 = orc.gradient(p, f, m, ffd, form=1, want_dDdM=True)
    assert D0 == D1
    assert np.abs(dm0 - dm1).max() <= 1e-12 * np.abs(dm0).max()
    assert np.linalg.norm(g0 - g1) <= 1e-12 * np.linalg.norm(g0)


@pytest.mark.parametrize("role", [0, 1])
def test_gradient_central_differences_16cube(orc, role):
    """Central differences of the oracle value on 16^3 smooth blobs (delta 5,
    7^3 control grid, K = 4, 32 bins, Phi ~ N(0, 1 vox), h = 1e-4)."""
    fr, mr = synth.smooth_pair((16, 16, 16), k=role)
    nb = 32
    f = orc.normalize(fr, fr.min(), fr.max(), nb)
    m = orc.normalize(mr, mr.min(), mr.max(), nb)
    p = P(orc, (16, 16, 16), nb=nb, K=(4, 4, 4), d=(5, 5, 5), role=role)
    ffd = synth.random_ffd(p.ctrl_dims, 1.0, 8 + role)
    D, g = orc.gradient(p, f, m, ffd)
    rng = np.random.default_rng(9)
    flat = np.argsort(-np.abs(g).ravel())
    idx = np.concatenate([flat[:60], rng.choice(flat[60:], 60, replace=False)])
    hstep = 1e-4
    fd = []
    for i in idx:
        e = np.zeros(g.size, dtype=np.float64)
        e[i] = hstep
        fp_ = (ffd.astype(np.float64).ravel() + e).astype(np.float32)
        fm_ = (ffd.astype(np.float64).ravel() - e).astype(np.float32)
        hh = (fp_.astype(np.float64) - fm_.astype(np.float64))[i]
        fd.append((orc.value(p, f, m, fp_.reshape(ffd.shape)) - orc.value(p, f, m, fm_.reshape(ffd.shape))) / hh)
    fd = np.array(fd)
    an = g.ravel()[idx]
    rel = np.linalg.norm(fd - an) / np.linalg.norm(an)
    assert rel < 1e-4, rel


# ------------------------------------------- dense displacement field
def _dense_from_ffd(orc, p, ffd):
    nx, ny, nz = p.fixed_dims
    u = np.zeros((3, nz, ny, nx), dtype=np.float64)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                u[:, z, y, x] = orc.ffd_T(p, ffd, x, y, z) - (x, y, z)
    return u.astype(np.float32)


@pytest.mark.parametrize("role", [0, 1])
def test_dense_field_chain_rule_to_ffd(orc, role):
    """A dense field sampled from an FFD gives the FFD's D, and eq 17 as the
    adjoint, sum_x beta_c(x) dD/du(x), gives the FFD gradient (beta from the
    centred cubic B-spline kernel)."""
    fr, mr = synth.smooth_pair((13, 12, 11), k=4 + role)
    nb = 24
    f = orc.normalize(fr, fr.min(), fr.max(), nb)
    m = orc.normalize(mr, mr.min(), mr.max(), nb)
    p = P(orc, (13, 12, 11), nb=nb, K=(4, 4, 4), d=(4, 4, 4), role=role)
    pd = orc.Problem(p.fixed_dims, p.moving_dims, nb, p.spatial_bins, p.ctrl_spacing, role, dense=True)
    ffd = synth.random_ffd(p.ctrl_dims, 0.8, 11)
    u = _dense_from_ffd(orc, p, ffd)
    D, g = orc.gradient(p, f, m, ffd)
    Dd, gd = orc.gradient(pd, f, m, u)
    assert gd.shape == (3, 11, 12, 13)
    assert abs(Dd - D) <= 1e-6 * D                     # u rounded to float32
    nx, ny, nz = p.fixed_dims
    ncx, ncy, ncz = p.ctrl_dims
    gc = np.zeros_like(g)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                pc = (x // 4, y // 4, z // 4)
                for n in range(4):
                    for mm in range(4):
                        for l in range(4):
                            b = (cubic_bspline_kernel(x / 4 - (pc[0] + l - 1)) * cubic_bspline_kernel(y / 4 - (pc[1] + mm - 1))
                                 * cubic_bspline_kernel(z / 4 - (pc[2] + n - 1)))
                            gc[:, pc[2] + n, pc[1] + mm, pc[0] + l] += b * gd[:, z, y, x]
    assert np.linalg.norm(gc - g) <= 1e-4 * np.linalg.norm(g)


def test_dense_gradient_central_differences(orc):
    """dD/du(x) of a dense field against central differences of D (h = 1e-3
    voxel) at voxels away from the grid edges."""
    fr, mr = synth.smooth_pair((14, 13, 12), k=6)
    nb = 24
    f = orc.normalize(fr, fr.min(), fr.max(), nb)
    m = orc.normalize(mr, mr.min(), mr.max(), nb)
    pd = orc.Problem((14, 13, 12), (14, 13, 12), nb, (4, 4, 4), (4, 4, 4), 0, dense=True)
    rng = np.random.default_rng(12)
    u = rng.normal(0.0, 0.7, size=(3, 12, 13, 14)).astype(np.float32)
    D, g = orc.gradient(pd, f, m, u)
    pts = [(int(rng.integers(3)), int(rng.integers(2, 10)), int(rng.integers(2, 11)), int(rng.integers(2, 12)))
           for _ in range(40)]
    fd = orc.fd_control_points(pd, f, m, u, pts, 1e-3)
    an = np.array([g[p_] for p_ in pts])
    assert np.linalg.norm(fd - an) <= 1e-3 * np.linalg.norm(an), (np.linalg.norm(fd - an) / np.linalg.norm(an))


# ------------------------------------------------ known stationary points
def test_zero_gradient_separated_levels_role_A(orc):
    """(Z-A): role A, piecewise-constant labels on non-integer bin positions at
    least 2 bins apart and B = f(A): every tap stays inside a one-bin-wide
    plateau of the regional means, so dD/dA = 0 at every voxel and the FFD
    gradient vanishes exactly at Phi = 0."""
    rng = np.random.default_rng(10)
    nx, ny, nz, nb = 12, 10, 9, 32
    levels = np.array([2.3, 6.6, 11.4, 17.8, 25.2])
    lab = (np.floor(np.arange(nx)[None, None, :] / 3) + np.floor(np.arange(ny)[None, :, None] / 4)
           + np.floor(np.arange(nz)[:, None, None] / 3)).astype(int) % len(levels)
    lab = np.broadcast_to(lab, (nz, ny, nx))
    A = levels[lab].astype(np.float32)
    B = levels[rng.permutation(len(levels))][lab].astype(np.float32)
    p = P(orc, (nx, ny, nz), nb=nb, K=(4, 4, 4), d=(3, 3, 3), role=0)
    ffd = np.zeros((3,) + p.ctrl_dims[::-1], dtype=np.float32)
    D, g = orc.gradient(p, B, A, ffd)
    assert D > 1e-6
    assert np.abs(g).max() < 1e-15


@pytest.mark.parametrize("role", [0, 1])
def test_mirror_ramp_gradient_symmetry(orc, role):
    """(Z-B): M a ramp along x, F an odd profile about the centre, lattices
    mirror-symmetric (delta | N-1): mirror + intensity flip is a symmetry, so
    g_y = g_z = 0 and g_x is antisymmetric under x -> mirror."""
    nx, ny, nz, nb = 26, 6, 6, 32
    xs = np.arange(nx, dtype=np.float64)
    # moving: s = 19/16 x + 21/32, exact in float32, never on a bin edge, and
    # L - s(x) = s(25 - x) exactly; linear in x, so one-sided trilinear
    # differences at the on-grid samples of Phi = 0 equal the two-sided ones
    ramp = np.broadcast_to((xs * 19.0 / 16.0 + 21.0 / 32.0)[None, None, :], (nz, ny, nx)).astype(np.float32)
    # fixed: an odd profile about the centre on a 1/256 grid, F(25 - x) = L - F(x) exactly
    half = np.round(256 * (15.5 + 15.5 * np.sin(np.pi * (xs[:13] - 12.5) / 25.0))) / 256.0
    prof = np.concatenate([half, 31.0 - half[::-1]])
    odd = np.broadcast_to(prof[None, None, :], (nz, ny, nx)).astype(np.float32)
    p = P(orc, (nx, ny, nz), nb=nb, K=(4, 4, 4), d=(5, 5, 5), role=role)
    ffd = np.zeros((3,) + p.ctrl_dims[::-1], dtype=np.float32)
    D, g = orc.gradient(p, odd, ramp, ffd)
    scale = np.abs(g[0]).max()
    assert scale > 1e-8
    assert np.abs(g[1]).max() <= 1e-12 * scale and np.abs(g[2]).max() <= 1e-12 * scale
    # stored node i sits at (i - 1) * delta; the mirror x -> (nx - 1) - x maps
    # node i to node (ncx - 2) - i; node ncx - 1 carries no weight at all.
    gx = g[0]
    n = gx.shape[2]
    assert np.abs(gx[:, :, n - 1]).max() == 0.0
    assert np.abs(gx[:, :, :n - 1] + gx[:, :, n - 2::-1]).max() <= 1e-12 * scale
    assert abs(gx.sum()) <= 1e-12 * np.abs(gx).sum()


@pytest.mark.parametrize("role", [0, 1])
def test_constant_estimated_image_closed_forms(orc, role):
    """B constant on a bin centre: sigma_r^2 = 0 in every region, all regions
    are degenerate and D = 0.  B constant off a bin centre: every voxel has the
    same two-bin Parzen distribution of B, no A-bin explains any of its
    variance (CR_r = 0) and D = sum_r p(r) = 1."""
    w = synth.blobs(n=14)
    nb = 32
    varying = orc.normalize(w.moving, w.moving.min(), w.moving.max(), nb)
    p = P(orc, (14, 14, 14), nb=nb, K=(4, 4, 4), d=(4, 4, 4), role=role)
    ffd = synth.random_ffd(p.ctrl_dims, 0.8, 23)
    for level, expect in ((7.0, 0.0), (7.25, 1.0)):
        const = np.full_like(varying, level)
        fixed, moving = (const, varying) if role == 0 else (varying, const)
        D, g = orc.gradient(p, fixed, moving, ffd)
        assert abs(D - expect) < 1e-12
        if expect == 0.0:
            assert np.abs(g).max() == 0.0


# ------------------------- regions on the FFD nodes (the paper's setting)
def test_node_weights_partition_and_interior_mass(orc):
    """Regions at the control points (Sec. II-C, eq 7 with eq 17's lattice):
    the weights of a voxel sum to 1, each is the centred cubic B-spline of
    the voxel's distance to its node in units of delta, and over the integer
    voxels of its whole support an interior node holds mass exactly delta."""
    N, d = 41, 5
    K = (N - 1) // d + 4
    tot = np.zeros(K)
    for x in range(N):
        w = orc.axis_node_weights(x, d, K)
        assert abs(w.sum() - 1.0) < 1e-15
        for j in range(K):                         # stored node j sits at (j - 1) delta
            assert abs(w[j] - cubic_bspline_kernel((x - (j - 1) * d) / d)) < 1e-15
        tot += w
    interior = range(3, N // d)                    # support ((j - 3) d, (j + 1) d) inside [0, N - 1]
    assert len(interior) >= 4
    for j in interior:
        assert abs(tot[j] - d) < 1e-12, (j, tot[j])


def test_node_regions_joint_pdf_marginal(orc):
    """p(r) of eq (3) with regions at the FFD nodes: Z = |Omega| and interior
    regions hold (delta^3 / Z) whatever the images."""
    nx, ny, nz, d = 26, 27, 21, 5
    p = orc.Problem((nx, ny, nz), (nx, ny, nz), 16, (0, 0, 0), (d, d, d), 0)
    fr, mr = synth.smooth_pair((nz, ny, nx), k=21)
    f = orc.normalize(fr, fr.min(), fr.max(), 16)
    m = orc.normalize(mr, mr.min(), mr.max(), 16)
    ffd = synth.random_ffd(p.ctrl_dims, 0.8, 22)
    pdf, Z = orc.joint_pdf(p, f, m, ffd)
    assert pdf.shape[0] == int(np.prod(p.ctrl_dims))
    assert abs(Z - nx * ny * nz) < 1e-9
    pr = pdf.sum(axis=(1, 2)).reshape(p.ctrl_dims[::-1]) * Z
    ncx, ncy, ncz = p.ctrl_dims
    inner = pr[3:nz // d, 3:ny // d, 3:nx // d]       # nodes whose whole support lies in the grid
    assert inner.size > 0 and np.allclose(inner, d ** 3, atol=1e-9)


@pytest.mark.parametrize("role", [0, 1])
def test_node_regions_D_zero_forms_and_gradient(orc, role):
    """Regions at the FFD nodes: D = 0 for B = f(A) on bin centres, the four
    value forms agree in [0, 1], and the gradient matches central differences."""
    rng = np.random.default_rng(23 + role)
    nx, ny, nz, nb = 13, 12, 11, 16
    labels = rng.integers(0, nb, size=(nz, ny, nx))
    A = labels.astype(np.float32)
    B = rng.permutation(nb)[labels].astype(np.float32)
    p = orc.Problem((nx, ny, nz), (nx, ny, nz), nb, (0, 0, 0), (4, 4, 4), role)
    fixed, moving = (B, A) if role == 0 else (A, B)
    assert abs(orc.value(p, fixed, moving, np.zeros((3,) + p.ctrl_dims[::-1], np.float32))) < 1e-14

    fr, mr = synth.smooth_pair((14, 14, 14), k=24 + role)
    nb = 24
    f = orc.normalize(fr, fr.min(), fr.max(), nb)
    m = orc.normalize(mr, mr.min(), mr.max(), nb)
    p = orc.Problem((14, 14, 14), (14, 14, 14), nb, (0, 0, 0), (5, 5, 5), role)
    ffd = synth.random_ffd(p.ctrl_dims, 0.8, 25 + role)
    pdf, _ = orc.joint_pdf(p, f, m, ffd)
    vals = [orc.srwcr_from_pdf(pdf, w) for w in range(4)]
    assert max(vals) - min(vals) < 1e-13 and 0.0 <= vals[0] <= 1.0
    D, g = orc.gradient(p, f, m, ffd)
    idx = np.argsort(-np.abs(g).ravel())[:40]
    fd = []
    for i in idx:
        fp_, fm_ = ffd.copy().ravel(), ffd.copy().ravel()
        fp_[i] = np.float32(float(ffd.ravel()[i]) + 1e-4)
        fm_[i] = np.float32(float(ffd.ravel()[i]) - 1e-4)
        hh = float(fp_[i]) - float(fm_[i])
        fd.append((orc.value(p, f, m, fp_.reshape(ffd.shape)) - orc.value(p, f, m, fm_.reshape(ffd.shape))) / hh)
    fd = np.array(fd)
    an = g.ravel()[idx]
    assert np.linalg.norm(fd - an) <= 1e-4 * np.linalg.norm(an)


# ------------------------------- derivative with respect to the fixed image
@pytest.mark.parametrize("role", [0, 1])
def test_fixed_image_gradient_central_differences(orc, role):
    """dD/ds_F per voxel (eq 19 or 21 for the fixed image's role) against
    central differences of D in single fixed voxels, and eqs 19/21 against
    eqs 18/20 with (26)."""
    fr, mr = synth.smooth_pair((12, 13, 14), k=30 + role)
    nb = 24
    f = orc.normalize(fr, fr.min(), fr.max(), nb)
    m = orc.normalize(mr, mr.min(), mr.max(), nb)
    p = P(orc, (14, 13, 12), nb=nb, K=(4, 4, 4), d=(5, 5, 5), role=role)
    ffd = synth.random_ffd(p.ctrl_dims, 0.8, 31 + role)
    D, g = orc.gradient_fixed(p, f, m, ffd)
    D1, g1 = orc.gradient_fixed(p, f, m, ffd, form=1)
    assert abs(D - orc.value(p, f, m, ffd)) < 1e-15 and abs(D1 - D) < 1e-15
    assert np.abs(g1 - g).max() <= 1e-12 * np.abs(g).max()
    idx = np.argsort(-np.abs(g).ravel())[:40]
    fd = []
    for i in idx:
        fp_, fm_ = f.copy().ravel(), f.copy().ravel()
        fp_[i] = np.float32(float(f.ravel()[i]) + 1e-3)
        fm_[i] = np.float32(float(f.ravel()[i]) - 1e-3)
        hh = float(fp_[i]) - float(fm_[i])
        fd.append((orc.value(p, fp_.reshape(f.shape), m, ffd) - orc.value(p, fm_.reshape(f.shape), m, ffd)) / hh)
    fd = np.array(fd)
    an = g.ravel()[idx]
    assert np.linalg.norm(fd - an) <= 1e-4 * np.linalg.norm(an), np.linalg.norm(fd - an) / np.linalg.norm(an)


def test_fixed_image_gradient_is_the_swapped_moving_gradient(orc):
    """With the identity warp and equal grids, the pair (fixed F, moving M,
    moving as A) has the same A and B as (fixed M, moving F, moving as B), so
    dD/ds_F of the first equals dD/ds_M of the second."""
    fr, mr = synth.smooth_pair((12, 12, 12), k=33)
    nb = 24
    f = orc.normalize(fr, fr.min(), fr.max(), nb)
    m = orc.normalize(mr, mr.min(), mr.max(), nb)
    p0 = P(orc, (12, 12, 12), nb=nb, K=(4, 4, 4), d=(4, 4, 4), role=0)
    p1 = P(orc, (12, 12, 12), nb=nb, K=(4, 4, 4), d=(4, 4, 4), role=1)
    zero = np.zeros((3,) + p0.ctrl_dims[::-1], np.float32)
    D0, gF = orc.gradient_fixed(p0, f, m, zero)
    D1, _, gM = orc.gradient(p1, m, f, zero, want_dDdM=True)
    assert abs(D0 - D1) < 1e-14
    assert np.abs(gF - gM).max() <= 1e-12 * np.abs(gM).max()
