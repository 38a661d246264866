"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Gates (spec tolerances): SRWCR value within 1e-5 relative, gradient
within 1e-4 relative L2, normalised intensities and fixed-image bins
bit-exact.  Inputs are seeded synthetic volumes; sizes span several work
items, ragged tails, unequal fixed / moving grids and both roles.
"""
import numpy as np
import pytest

from workloads import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

VALUE_TOL = 1e-5
GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def S():
    import paper_1804_05061_amd as S
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return S


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def prepare(S, orc, fixed_raw, moving_raw, nb, K, delta, role, fdt=0, mdt=0):
    fl, fh = float(fixed_raw.min()), float(fixed_raw.max())
    ml, mh = float(moving_raw.min()), float(moving_raw.max())
    tdt = {0: torch.float32, 1: torch.float16, 2: torch.bfloat16}
    f_g = S.normalize(dev(fixed_raw), fl, fh, nb, tdt[fdt])
    m_g = S.normalize(dev(moving_raw), ml, mh, nb, tdt[mdt])
    fdims = tuple(fixed_raw.shape[::-1])
    mdims = tuple(moving_raw.shape[::-1])
    prob = S.Problem(fdims, mdims, nb, K, delta, role, fdt, mdt)
    P = orc.Problem(fdims, mdims, nb, K, delta, role)
    # the oracle sees exactly the stored (possibly 16-bit) normalised values
    f_o = f_g.float().cpu().numpy()
    m_o = m_g.float().cpu().numpy()
    return prob, P, f_g, m_g, f_o, m_o


def oracle_moments(orc, P, f, m, ffd):
    pdf, Z = orc.joint_pdf(P, f, m, ffd)
    b = np.arange(P.n_bins, dtype=np.float64)
    return np.stack([pdf.sum(2) * Z, (pdf * b).sum(2) * Z, (pdf * b * b).sum(2) * Z], axis=-1)


def check_value_grad(S, orc, prob, P, f_g, m_g, f_o, m_o, ffd, label=""):
    plan = S.Plan(prob)
    D, g = plan.grad(f_g, m_g, dev(ffd))
    D2 = plan.eval(f_g, m_g, dev(ffd))
    torch.cuda.synchronize()
    D, D2, g = float(D.item()), float(D2.item()), g.cpu().numpy().astype(np.float64)
    Dr, gr = orc.gradient(P, f_o, m_o, ffd)
    rel_v = abs(D - Dr) / abs(Dr)
    rel_g = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    print(f"{label} items={plan.info()['n_items']} D={D:.12f} oracle={Dr:.12f} rel={rel_v:.2e} "
          f"grad relL2={rel_g:.2e}", flush=True)
    # the cross-workgroup FP64 merge is atomic, so its summation order may vary
    assert abs(D - D2) <= 1e-12 * abs(D), "srwcr_eval and srwcr_grad disagree on D"
    assert rel_v <= VALUE_TOL, (label, D, Dr, rel_v)
    assert rel_g <= GRAD_TOL, (label, rel_g)
    return plan, D, g


def test_normalize_bit_exact_and_minmax(S, orc):
    w = synth.blobs(n=40)
    x = dev(w.fixed)
    lo, hi = S.minmax(x)
    assert lo == float(w.fixed.min()) and hi == float(w.fixed.max())
    for nb in (32, 64, 17):
        got = S.normalize(x, lo, hi, nb).cpu().numpy()
        assert np.array_equal(got, orc.normalize(w.fixed, lo, hi, nb))
    h16 = S.normalize(x, lo, hi, 64, torch.float16).cpu().numpy()
    ref = orc.normalize(w.fixed, lo, hi, 64)
    assert np.array_equal(h16, ref.astype(np.float16))
    b16 = S.normalize(x, lo, hi, 64, torch.bfloat16).float().cpu().numpy()
    assert np.array_equal(b16, torch.from_numpy(ref).to(torch.bfloat16).float().numpy())


@pytest.mark.parametrize("role", [0, 1])
def test_moments_blobs64(S, orc, role):
    w = synth.blobs()
    prob, P, f_g, m_g, f_o, m_o = prepare(S, orc, w.fixed, w.moving, 32, (4, 4, 4), (8, 8, 8), role)
    ffd = synth.random_ffd(prob.ctrl_dims, 1.0, 11)
    plan = S.Plan(prob)
    mg = plan.debug_moments(f_g, m_g, dev(ffd)).cpu().numpy()
    mo = oracle_moments(orc, P, f_o, m_o, ffd)
    err = np.abs(mg - mo) / (np.abs(mo).max(axis=(0, 1)) + 1e-30)
    print("moment rel err", err.max(axis=(0, 1)), flush=True)
    assert err.max() < 1e-6


@pytest.mark.parametrize("role", [0, 1])
def test_moments_nodes_ragged(S, orc, role):
    """Regions at the FFD nodes with unequal spacings (5, 4, 6) on a ragged
    grid: blocks of two small cells per axis, which the value pass sums per
    column on the matrix cores; the raw moments element by element against
    the oracle's eq (3) reduction."""
    w = synth.blobs(n=48)
    fixed = np.ascontiguousarray(w.fixed[:37, :43, :47])
    moving = np.ascontiguousarray(w.moving[:37, :43, :47])
    prob, P, f_g, m_g, f_o, m_o = prepare(S, orc, fixed, moving, 32, (0, 0, 0), (5, 4, 6), role)
    ffd = synth.random_ffd(prob.ctrl_dims, 1.2, 14)
    plan = S.Plan(prob)
    mg = plan.debug_moments(f_g, m_g, dev(ffd)).cpu().numpy()
    mo = oracle_moments(orc, P, f_o, m_o, ffd)
    err = np.abs(mg - mo) / (np.abs(mo).max(axis=(0, 1)) + 1e-30)
    print("nodes moment rel err", err.max(axis=(0, 1)), flush=True)
    assert err.max() < 1e-6


@pytest.mark.parametrize("role", [0, 1])
@pytest.mark.parametrize("sigma", [0.0, 1.0])
def test_blobs64_value_and_gradient(S, orc, role, sigma):
    """Workload 1: 64^3 blobs, 32 bins, 4x4x4 regions, FFD spacing 8."""
    w = synth.blobs()
    prob, P, f_g, m_g, f_o, m_o = prepare(S, orc, w.fixed, w.moving, 32, (4, 4, 4), (8, 8, 8), role)
    ffd = synth.random_ffd(prob.ctrl_dims, sigma, 12) if sigma else np.zeros(prob.ffd_shape, np.float32)
    check_value_grad(S, orc, prob, P, f_g, m_g, f_o, m_o, ffd, f"blobs64 role={role} sigma={sigma}")


@pytest.mark.parametrize("role", [0, 1])
def test_ragged_grid(S, orc, role):
    """Odd sizes: ragged row segments, cells of unequal width, 24 bins."""
    w = synth.blobs(n=48)
    fixed = np.ascontiguousarray(w.fixed[:23, :29, :37])
    moving = np.ascontiguousarray(w.moving[:23, :29, :37])
    prob, P, f_g, m_g, f_o, m_o = prepare(S, orc, fixed, moving, 24, (5, 4, 6), (3, 4, 5), role)
    ffd = synth.random_ffd(prob.ctrl_dims, 0.8, 13)
    check_value_grad(S, orc, prob, P, f_g, m_g, f_o, m_o, ffd, f"ragged role={role}")


@pytest.mark.parametrize("role", [0, 1])
def test_unequal_grids(S, orc, role):
    """Moving grid half the fixed grid (the CT/PET set-up of workload 4, small)."""
    w = synth.blobs(n=40)
    fixed = w.fixed[:32, :36, :40]
    moving = np.ascontiguousarray(w.moving[:32:2, :36:2, :40:2])
    prob, P, f_g, m_g, f_o, m_o = prepare(S, orc, np.ascontiguousarray(fixed), moving, 48, (5, 5, 5), (8, 8, 8),
                                          role)
    ffd = synth.random_ffd(prob.ctrl_dims, 1.5, 14)
    check_value_grad(S, orc, prob, P, f_g, m_g, f_o, m_o, ffd, f"unequal role={role}")


def test_ffd_warp_matches_oracle(S, orc):
    w = synth.blobs(n=40)
    fixed = np.ascontiguousarray(w.fixed[:31, :35, :40])
    moving = np.ascontiguousarray(w.moving[:31, :35, :40])
    prob, P, f_g, m_g, f_o, m_o = prepare(S, orc, fixed, moving, 32, (4, 4, 4), (5, 5, 5), 0)
    ffd = synth.random_ffd(prob.ctrl_dims, 3.0, 15)     # large enough to push samples off the grid
    plan = S.Plan(prob)
    got = plan.warp(m_g, dev(ffd)).cpu().numpy().astype(np.float64)
    ref = orc.warp(P, m_o, ffd)
    # FP64 arithmetic on both sides (different operation order), rounded once
    # to FP32 on the GPU: within one FP32 unit in the last place of the oracle
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    err = np.abs(got - ref)
    print(f"warp: max |err| {err.max():.3e}, max err / ulp {(err / ulp).max():.3f}", flush=True)
    assert np.all(err <= ulp)
    zero = plan.warp(m_g, dev(np.zeros_like(ffd))).cpu().numpy()
    assert np.array_equal(zero, m_o)


def check_bins(S, orc, plan, P, m_g, m_o, ffd, label):
    """The hot path's moving bin k = min(floor(s), L - 1) of every fixed voxel
    (eq 5), as the value and gradient passes read it, against the oracle's
    warped sample s; and the in-bin position s - k against the oracle's,
    rounded to FP32.  Both sides decide k in FP64, so a mismatch can only come
    from a sample within rounding distance of a bin edge: each one is counted
    and must lie within 1e-9 bins of the edge.  The two FP64 evaluations of s
    differ in operation order by a few FP64 units of |s| <= L (~1e-14); where
    t is near 0 that exceeds the FP32 unit of t, so t is held to one FP32 unit
    plus 1e-12."""
    k_g, t_g = plan.debug_samples(m_g, dev(ffd))
    k_g = k_g.cpu().numpy()
    t_g = t_g.cpu().numpy().astype(np.float64)
    s = orc.warp(P, m_o, ffd)
    L = P.n_bins - 1
    k_o = np.minimum(np.floor(s), L - 1).astype(np.int32)
    mism = k_g != k_o
    n_mism = int(mism.sum())
    edge = np.abs(s - np.round(s))
    print(f"{label}: {k_g.size} voxels, {n_mism} bin mismatches, nearest sample to a bin edge "
          f"{edge.min():.2e} bins", flush=True)
    assert np.all(edge[mism] <= 1e-9)
    t_o = s - k_o
    ok = ~mism
    ulp = np.spacing(np.abs(t_o[ok]).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(t_g[ok] - t_o[ok]) <= ulp + 1e-12)
    return n_mism


@pytest.mark.parametrize("case", ["blobs64", "ragged", "unequal"])
def test_warped_bins_match_oracle(S, orc, case):
    w = synth.blobs(n=64 if case == "blobs64" else 48)
    if case == "blobs64":
        fixed, moving, nb, K, d = w.fixed, w.moving, 32, (4, 4, 4), (8, 8, 8)
    elif case == "ragged":
        fixed = np.ascontiguousarray(w.fixed[:23, :29, :37])
        moving = np.ascontiguousarray(w.moving[:23, :29, :37])
        nb, K, d = 24, (5, 4, 6), (3, 4, 5)
    else:
        fixed = np.ascontiguousarray(w.fixed[:32, :36, :40])
        moving = np.ascontiguousarray(w.moving[:32:2, :36:2, :40:2])
        nb, K, d = 48, (5, 5, 5), (8, 8, 8)
    prob, P, f_g, m_g, f_o, m_o = prepare(S, orc, fixed, moving, nb, K, d, 0)
    plan = S.Plan(prob)
    for sigma, seed in ((0.0, 0), (1.5, 19), (3.0, 20)):
        ffd = synth.random_ffd(prob.ctrl_dims, sigma, seed) if sigma else np.zeros(prob.ffd_shape, np.float32)
        assert check_bins(S, orc, plan, P, m_g, m_o, ffd, f"{case} sigma={sigma}") == 0


def test_invalid_arguments_raise(S):
    with pytest.raises(S.SrwcrError):
        S.Plan(S.Problem((1, 8, 8), (8, 8, 8), 32, (4, 4, 4), (4, 4, 4)))
    with pytest.raises(S.SrwcrError):
        S.Plan(S.Problem((8, 8, 8), (8, 8, 8), 65, (4, 4, 4), (4, 4, 4)))
    with pytest.raises(S.SrwcrError):
        S.Plan(S.Problem((8, 8, 8), (8, 8, 8), 32, (3, 4, 4), (4, 4, 4)))
    with pytest.raises(S.SrwcrError):
        S.Plan(S.Problem((8, 8, 8), (8, 8, 8), 32, (4, 4, 4), (0, 4, 4)))
    with pytest.raises(S.SrwcrError):
        S.normalize(dev(np.ones(10, np.float32)), 1.0, 1.0, 32)
    x = np.ones(1000, np.float32)
    x[7] = np.nan
    with pytest.raises(S.SrwcrError):
        S.minmax(dev(x))


@pytest.mark.parametrize("role", [0, 1])
def test_narrow_cells_and_unit_spacing(S, orc, role):
    """Spatial cells narrower than a wave (x chunks of two cells, partial
    segments) and FFD spacing 1 (the widest control support per segment)."""
    w = synth.blobs(n=40)
    fixed = np.ascontiguousarray(w.fixed[:20, :30, :40])
    moving = np.ascontiguousarray(w.moving[:20, :30, :40])
    prob, P, f_g, m_g, f_o, m_o = prepare(S, orc, fixed, moving, 16, (10, 8, 6), (1, 3, 2), role)
    ffd = synth.random_ffd(prob.ctrl_dims, 0.3, 16)
    check_value_grad(S, orc, prob, P, f_g, m_g, f_o, m_o, ffd, f"narrow role={role}")


def test_two_bins(S, orc):
    """L_eps = 1: every tap lands on bins 0 and 1."""
    w = synth.blobs(n=24)
    prob, P, f_g, m_g, f_o, m_o = prepare(S, orc, w.fixed, w.moving, 2, (4, 4, 4), (6, 6, 6), 0)
    ffd = synth.random_ffd(prob.ctrl_dims, 1.0, 17)
    check_value_grad(S, orc, prob, P, f_g, m_g, f_o, m_o, ffd, "two bins")


@pytest.mark.parametrize("role", [0, 1])
def test_constant_estimated_image(S, orc, role):
    """A constant estimated image B on a bin centre has sigma_r^2 = 0 in every
    region: all regions are skipped, D = 0 and the gradient vanishes.  Off a
    bin centre the Parzen window (eq 5) spreads it over two bins: sigma_r^2 =
    w0 w1 > 0, no A-bin explains any of it, and D = 1 exactly."""
    w = synth.blobs(n=24)
    nb = 32
    lo, hi = float(w.moving.min()), float(w.moving.max())
    varying = S.normalize(dev(w.moving), lo, hi, nb)
    prob = S.Problem(w.fixed_dims, w.moving_dims, nb, (4, 4, 4), (6, 6, 6), role)
    ffd_np = synth.random_ffd(prob.ctrl_dims, 1.0, 18)
    ffd = dev(ffd_np)
    plan = S.Plan(prob)
    for level, expect in ((7.0, 0.0), (7.25, 1.0)):
        const = torch.full_like(varying, level)
        fixed, moving = (const, varying) if role == 0 else (varying, const)
        D, g = plan.grad(fixed, moving, ffd)
        torch.cuda.synchronize()
        P = orc.Problem(prob.fixed_dims, prob.moving_dims, nb, (4, 4, 4), (6, 6, 6), role)
        Dr, gr = orc.gradient(P, fixed.cpu().numpy(), moving.cpu().numpy(), ffd_np)
        assert abs(Dr - expect) < 1e-12
        assert abs(float(D.item()) - expect) < 1e-6, (level, float(D.item()))
        if expect == 0.0:
            assert float(g.abs().max().item()) == 0.0
        gg = g.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(gg - gr) <= GRAD_TOL * max(np.linalg.norm(gr), 1e-12) + 1e-12


def test_repeated_calls_on_one_workspace(S, orc):
    """Calls in a row on one plan and workspace start clean: an FFD gradient
    that follows another FFD gradient, a dense-field gradient and a value call
    matches the oracle for its own input (a plan whose value pass is staged
    clears the FFD gradient accumulators inside the warp pass)."""
    w = synth.blobs()
    prob, P, f_g, m_g, f_o, m_o = prepare(S, orc, w.fixed, w.moving, 32, (4, 4, 4), (8, 8, 8), 0)
    plan = S.Plan(prob)
    field = dev(np.zeros((3,) + w.fixed.shape, np.float32))
    ffds = [synth.random_ffd(prob.ctrl_dims, 1.0, 21), synth.random_ffd(prob.ctrl_dims, 1.0, 22)]
    for i, ffd in enumerate(ffds):
        plan.grad(f_g, m_g, dev(ffds[1 - i]))
        plan.grad_dense(f_g, m_g, field)
        plan.eval(f_g, m_g, dev(ffds[1 - i]))
        D, g = plan.grad(f_g, m_g, dev(ffd))
        torch.cuda.synchronize()
        D, g = float(D.item()), g.cpu().numpy().astype(np.float64)
        Dr, gr = orc.gradient(P, f_o, m_o, ffd)
        rel_v, rel_g = abs(D - Dr) / abs(Dr), np.linalg.norm(g - gr) / np.linalg.norm(gr)
        print(f"call {i}: D rel={rel_v:.2e} grad relL2={rel_g:.2e}", flush=True)
        assert rel_v <= VALUE_TOL and rel_g <= GRAD_TOL, (i, rel_v, rel_g)


def test_profile_modes(S):
    """HIP-event timing: mode 1 times every phase, modes 2 and 3 only the
    value pass and only the gradient pass; a mode outside 0..3 is refused.
    Timing does not change the results."""
    w = synth.blobs()
    nb = 32
    prob = S.Problem(w.fixed_dims, w.moving_dims, nb, (4, 4, 4), (8, 8, 8), S.MOVING_AS_A)
    f = S.normalize(dev(w.fixed), float(w.fixed.min()), float(w.fixed.max()), nb)
    m = S.normalize(dev(w.moving), float(w.moving.min()), float(w.moving.max()), nb)
    ffd = dev(synth.random_ffd(prob.ctrl_dims, 1.0, 23))
    plan = S.Plan(prob)
    D0, g0 = plan.grad(f, m, ffd)
    for mode, timed in ((1, {"warp", "value", "finalize", "grad", "grad_out"}), (2, {"value"}), (3, {"grad"})):
        plan.profile(mode)
        for _ in range(3):
            D, g = plan.grad(f, m, ffd)
        r = plan.profile_read()
        plan.profile(0)
        print(mode, r, flush=True)
        assert r["calls"] == 3
        for k in ("warp", "value", "finalize", "grad", "grad_out"):
            assert (r[k] > 0) == (k in timed), (mode, k, r)
        assert float(D.item()) == float(D0.item()) or abs(float(D.item()) - float(D0.item())) <= 1e-12
        assert torch.allclose(g, g0, rtol=1e-5, atol=1e-9)
    with pytest.raises(S.SrwcrError, match="INVALID_ARG"):
        plan.profile(4)
