"""RaPTOR (eqs 6, 13, 14) on the GPU against the FP64 oracle: value and
gradient for the FFD and a dense field in both roles on a ragged grid with
clipped, empty and whole-grid patches, the full 256x256x128 CT workload, and
the argument checks of the C ABI."""
import numpy as np
import pytest

from workloads import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def small_case(S, orc, role, dense):
    dims = (70, 45, 23)                                       # (nx, ny, nz): a ragged x tail past 64
    fr, mr = synth.smooth_pair(dims[::-1], k=40 + role, n_blobs=10)
    nb = 32
    P = S.Problem(dims, dims, nb, (4, 4, 4), (5, 5, 5), role)
    f = S.normalize(torch.from_numpy(fr).cuda(), float(fr.min()), float(fr.max()), nb)
    m = S.normalize(torch.from_numpy(mr).cuda(), float(mr.min()), float(mr.max()), nb)
    if dense:
        rng = np.random.default_rng(1804_05061 + 90 + role)
        disp = rng.normal(0.0, 0.8, size=P.field_shape).astype(np.float32)
    else:
        disp = synth.random_ffd(P.ctrl_dims, 1.0, 41 + role)
    boxes = synth.raptor_patches(dims, side=9, coverage=1.5, k=42 + role)
    Po = orc.Problem(dims, dims, nb, (4, 4, 4), (5, 5, 5), role, dense=dense)
    fo = orc.normalize(fr, float(fr.min()), float(fr.max()), nb)
    mo = orc.normalize(mr, float(mr.min()), float(mr.max()), nb)
    return P, f, m, disp, boxes, Po, fo, mo


@pytest.mark.parametrize("role", [0, 1])
@pytest.mark.parametrize("dense", [False, True])
def test_raptor_matches_oracle(orc, role, dense):
    import paper_1804_05061_amd as S
    P, f, m, disp, boxes, Po, fo, mo = small_case(S, orc, role, dense)
    plan = S.Plan(P)
    rp = S.RaptorPatches(plan, boxes)
    d = torch.from_numpy(disp).cuda()
    v, g = rp.grad(f, m, d, dense=dense)
    ve = rp.eval(f, m, d, dense=dense)
    torch.cuda.synchronize()
    vr, gr = orc.raptor(Po, fo, mo, disp, boxes, want_grad=True)
    gg = g.cpu().numpy().astype(np.float64)
    print(f"raptor role={role} dense={dense}: {float(v):.12f} oracle {vr:.12f} "
          f"(rel {abs(float(v) - vr) / vr:.1e}); grad rel {rel(gg, gr):.2e}", flush=True)
    assert abs(float(v) - vr) <= 1e-5 * vr
    assert abs(float(ve) - float(v)) <= 1e-12 * vr
    assert rel(gg, gr) <= 1e-4
    # a second call on the same workspace gives the same result
    v2, g2 = rp.grad(f, m, d, dense=dense)
    torch.cuda.synchronize()
    assert abs(float(v2) - float(v)) <= 1e-12 * vr
    assert rel(g2.cpu().numpy(), gg) <= 1e-6


@pytest.mark.parametrize("edge", [False, True])
def test_raptor_ct256_full_size(orc, edge):
    """256x256x128 CT phantom, 64 bins, ~1.0x coverage by 17^3 patches (the
    benchmark's set; with `edge`, plus a patch outside the grid and one over
    all of it): value and FFD gradient of the whole workload against the oracle."""
    import paper_1804_05061_amd as S
    w = synth.ct_phantom()
    fr, mr = w.fixed, w.moving
    P = S.Problem(w.fixed_dims, w.moving_dims, w.n_bins, w.spatial_bins, w.ctrl_spacing, w.role)
    flo, fhi = float(fr.min()), float(fr.max())
    mlo, mhi = float(mr.min()), float(mr.max())
    f = S.normalize(torch.from_numpy(fr).cuda(), flo, fhi, w.n_bins)
    m = S.normalize(torch.from_numpy(mr).cuda(), mlo, mhi, w.n_bins)
    ffd = synth.random_ffd(P.ctrl_dims, 1.5, 43)
    boxes = synth.raptor_patches(w.fixed_dims, side=17, coverage=1.0, k=44, extra_edge=edge)
    plan = S.Plan(P)
    rp = S.RaptorPatches(plan, boxes)
    v, g = rp.grad(f, m, torch.from_numpy(ffd).cuda())
    torch.cuda.synchronize()
    Po = orc.Problem(w.fixed_dims, w.moving_dims, w.n_bins, w.spatial_bins, w.ctrl_spacing, w.role)
    fo = orc.normalize(fr, flo, fhi, w.n_bins)
    mo = orc.normalize(mr, mlo, mhi, w.n_bins)
    vr, gr = orc.raptor(Po, fo, mo, ffd, boxes, want_grad=True)
    gg = g.cpu().numpy().astype(np.float64)
    print(f"raptor ct256 edge={edge} ({len(boxes)} patches): {float(v):.12f} oracle {vr:.12f} "
          f"(rel {abs(float(v) - vr) / vr:.1e}); grad rel {rel(gg, gr):.2e}", flush=True)
    assert abs(float(v) - vr) <= 1e-5 * vr
    assert rel(gg, gr) <= 1e-4


def test_raptor_argument_checks():
    import paper_1804_05061_amd as S
    dims = (20, 18, 16)
    P = S.Problem(dims, dims, 16, (4, 4, 4), (5, 5, 5), 0)
    plan, other = S.Plan(P), S.Plan(P)
    with pytest.raises(S.SrwcrError, match="INVALID_ARG"):
        S.RaptorPatches(plan, np.zeros((0, 6), dtype=np.int32))
    rp = S.RaptorPatches(plan, [[0, 0, 0, 8, 8, 8]])
    f = torch.zeros(P.fixed_shape, device="cuda")
    m = torch.zeros(P.moving_shape, device="cuda")
    d = torch.zeros(P.ffd_shape, device="cuda")
    out = torch.empty((), dtype=torch.float64, device="cuda")
    L = S._lib.load()
    p = S._ptr
    # a patch set made for another plan
    st = L.raptor_eval(other.handle, rp._h, p(f), p(m), p(d), 0, p(out), p(rp.workspace), rp.workspace_bytes,
                       S._stream())
    assert st == -1 and b"another plan" in L.srwcr_last_error()
    assert L.raptor_workspace_bytes(other.handle, rp._h) == 0
    # workspace too small
    st = L.raptor_eval(plan.handle, rp._h, p(f), p(m), p(d), 0, p(out), p(rp.workspace), rp.workspace_bytes - 1,
                       S._stream())
    assert st == -3
    # dense flag out of range
    st = L.raptor_eval(plan.handle, rp._h, p(f), p(m), p(d), 2, p(out), p(rp.workspace), rp.workspace_bytes,
                       S._stream())
    assert st == -1
    # constant B: every patch is skipped and RaPTOR is 0
    v = rp.eval(f, m, d)
    torch.cuda.synchronize()
    assert float(v) == 0.0


@pytest.mark.parametrize("fdt,mdt,role", [(1, 1, 0), (2, 2, 1), (1, 0, 1)])
def test_raptor_and_fixed_gradient_16bit_storage(orc, fdt, mdt, role):
    """FP16 / BF16 storage of the normalised volumes: RaPTOR (value and FFD
    gradient) and dD/ds_F against the oracle run on the same stored values."""
    import paper_1804_05061_amd as S
    tdt = {0: torch.float32, 1: torch.float16, 2: torch.bfloat16}
    dims = (70, 45, 23)
    fr, mr = synth.smooth_pair(dims[::-1], k=50 + fdt + mdt, n_blobs=10)
    nb = 32
    f = S.normalize(torch.from_numpy(fr).cuda(), float(fr.min()), float(fr.max()), nb, tdt[fdt])
    m = S.normalize(torch.from_numpy(mr).cuda(), float(mr.min()), float(mr.max()), nb, tdt[mdt])
    fo, mo = f.float().cpu().numpy(), m.float().cpu().numpy()     # the stored values, exactly
    P = S.Problem(dims, dims, nb, (4, 4, 4), (5, 5, 5), role, fdt, mdt)
    plan = S.Plan(P)
    ffd = synth.random_ffd(P.ctrl_dims, 1.0, 51 + role)
    boxes = synth.raptor_patches(dims, side=9, coverage=1.5, k=52)
    rp = S.RaptorPatches(plan, boxes)
    v, g = rp.grad(f, m, torch.from_numpy(ffd).cuda())
    D, gF = plan.grad_fixed(f, m, torch.from_numpy(ffd).cuda())
    torch.cuda.synchronize()
    Po = orc.Problem(dims, dims, nb, (4, 4, 4), (5, 5, 5), role)
    vr, gr = orc.raptor(Po, fo, mo, ffd, boxes, want_grad=True)
    Dr, gFr = orc.gradient_fixed(Po, fo, mo, ffd)
    print(f"16-bit fdt={fdt} mdt={mdt} role={role}: RaPTOR rel {abs(float(v) - vr) / vr:.1e} grad "
          f"{rel(g.cpu().numpy(), gr):.2e}; D rel {abs(float(D) - Dr) / Dr:.1e} dD/dF {rel(gF.cpu().numpy(), gFr):.2e}",
          flush=True)
    assert abs(float(v) - vr) <= 1e-5 * vr and rel(g.cpu().numpy(), gr) <= 1e-4
    assert abs(float(D) - Dr) <= 1e-5 * Dr and rel(gF.cpu().numpy(), gFr) <= 1e-4
