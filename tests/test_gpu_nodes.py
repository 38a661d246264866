"""Regions at the FFD nodes (the paper's own setting, Sec. II-C: delta_s =
delta = 5, 32 bins): value and gradient against the FP64 oracle on a small
grid in both roles, and at the paper's 256 x 256 x 99 operating point."""
import numpy as np
import pytest

from workloads import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def run_pair(S, orc, fr, mr, nb, delta, role, ffd_sigma, seed, dense=False):
    dims = tuple(int(v) for v in fr.shape[::-1])
    P = S.Problem(dims, dims, nb, (0, 0, 0), (delta,) * 3, role)
    flo, fhi, mlo, mhi = float(fr.min()), float(fr.max()), float(mr.min()), float(mr.max())
    f = S.normalize(torch.from_numpy(fr).cuda(), flo, fhi, nb)
    m = S.normalize(torch.from_numpy(mr).cuda(), mlo, mhi, nb)
    ffd = synth.random_ffd(P.ctrl_dims, ffd_sigma, seed)
    plan = S.Plan(P)
    D, g = plan.grad(f, m, torch.from_numpy(ffd).cuda())
    De = plan.eval(f, m, torch.from_numpy(ffd).cuda())
    torch.cuda.synchronize()
    Po = orc.Problem(dims, dims, nb, (0, 0, 0), (delta,) * 3, role)
    fo = orc.normalize(fr, flo, fhi, nb)
    mo = orc.normalize(mr, mlo, mhi, nb)
    Dr, gr = orc.gradient(Po, fo, mo, ffd)
    return float(D), float(De), g.cpu().numpy().astype(np.float64), Dr, gr, P


@pytest.mark.parametrize("role", [0, 1])
def test_node_regions_match_oracle_blobs(orc, role):
    import paper_1804_05061_amd as S
    w = synth.blobs(64)
    D, De, g, Dr, gr, P = run_pair(S, orc, w.fixed, w.moving, 32, 5, role, 1.0, 61 + role)
    print(f"nodes blobs64 role={role} ({P.n_regions} regions): D={D:.12f} oracle={Dr:.12f} "
          f"(rel {abs(D - Dr) / Dr:.1e}); grad rel {rel(g, gr):.2e}", flush=True)
    assert abs(D - Dr) <= 1e-5 * Dr
    assert abs(De - D) <= 1e-12 * Dr
    assert rel(g, gr) <= 1e-4


def test_node_regions_paper_operating_point(orc):
    """256 x 256 x 99 CT-like phantom, 32 bins, regions = FFD nodes at delta 5
    (55 x 55 x 23 = 69,575 regions), moving as A, Phi ~ N(0, 1.5 vox)."""
    import paper_1804_05061_amd as S
    w = synth.ct_phantom(shape=(99, 256, 256))
    D, De, g, Dr, gr, P = run_pair(S, orc, w.fixed, w.moving, 32, 5, 0, 1.5, 51)
    print(f"nodes ct256x99 ({P.n_regions} regions): D={D:.12f} oracle={Dr:.12f} "
          f"(rel {abs(D - Dr) / Dr:.1e}); grad rel {rel(g, gr):.2e}", flush=True)
    assert P.n_regions == 55 * 55 * 23
    assert abs(D - Dr) <= 1e-5 * Dr
    assert rel(g, gr) <= 1e-4
