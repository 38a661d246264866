"""srwcr_grad_batched: independent problems of different sizes (breathing
phases x pyramid levels) evaluated by one launch per pass, checked problem by
problem against the FP64 oracle and against single-plan srwcr_grad, eagerly and
through replays of a captured HIP graph."""
import numpy as np
import pytest
from scipy import ndimage

from workloads import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NB, K, DELTA = 32, (4, 4, 4), (6, 6, 6)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def levels(vol, n):
    """Pyramid of a raw volume: Gaussian sigma = 1 voxel, then every second voxel."""
    out = [vol]
    for _ in range(n - 1):
        out.append(np.ascontiguousarray(ndimage.gaussian_filter(out[-1], 1.0)[::2, ::2, ::2]))
    return out


@pytest.fixture(scope="module")
def problems():
    import paper_1804_05061_amd as S
    pairs = synth.breathing_phases(shape=(40, 72, 64), n_phases=3)
    out = []
    for pi, (f_raw, m_raw) in enumerate(pairs):
        flo, fhi, mlo, mhi = f_raw.min(), f_raw.max(), m_raw.min(), m_raw.max()
        for lv, (f_l, m_l) in enumerate(zip(levels(f_raw, 2), levels(m_raw, 2))):
            nz, ny, nx = f_l.shape
            prob = S.Problem((nx, ny, nz), (nx, ny, nz), NB, K, DELTA, S.MOVING_AS_A)
            ffd = synth.random_ffd(prob.ctrl_dims, 1.5, 50 + 3 * pi + lv)
            f = S.normalize(torch.from_numpy(f_l).cuda(), flo, fhi, NB)
            m = S.normalize(torch.from_numpy(m_l).cuda(), mlo, mhi, NB)
            out.append(dict(prob=prob, plan=S.Plan(prob), f=f, m=m, ffd=torch.from_numpy(ffd).cuda(), ffd_np=ffd,
                            f_raw=f_l, m_raw=m_l, rng=(flo, fhi, mlo, mhi)))
    return out


def test_batched_matches_oracle_and_single_plans(orc, problems):
    import paper_1804_05061_amd as S
    batch = S.Batch([p["plan"] for p in problems])
    vals, grads = batch.grad([(p["f"], p["m"], p["ffd"]) for p in problems])
    torch.cuda.synchronize()
    for i, p in enumerate(problems):
        D1, g1 = p["plan"].grad(p["f"], p["m"], p["ffd"])
        flo, fhi, mlo, mhi = p["rng"]
        pr = p["prob"]
        P = orc.Problem(pr.fixed_dims, pr.moving_dims, NB, K, DELTA, 0)
        fo = orc.normalize(p["f_raw"], flo, fhi, NB)
        mo = orc.normalize(p["m_raw"], mlo, mhi, NB)
        Dr, gr = orc.gradient(P, fo, mo, p["ffd_np"])
        Db, gb = float(vals[i]), grads[i].cpu().numpy().astype(np.float64)
        print(f"problem {i} {pr.fixed_dims}: D={Db:.12f} oracle={Dr:.12f} single={float(D1):.12f} "
              f"grad vs oracle {rel(gb, gr):.2e} vs single {rel(gb, g1.cpu().numpy()):.2e}", flush=True)
        assert abs(Db - Dr) <= 1e-5 * abs(Dr)
        assert rel(gb, gr) <= 1e-4
        assert abs(Db - float(D1)) <= 1e-12 * abs(Dr)            # same arithmetic, other atomic order
        assert rel(gb, g1.cpu().numpy()) <= 1e-6


def test_batched_graph_replays(problems):
    import paper_1804_05061_amd as S
    batch = S.Batch([p["plan"] for p in problems])
    inputs = [(p["f"], p["m"], p["ffd"].clone()) for p in problems]
    vals = torch.empty(len(problems), dtype=torch.float64, device="cuda")
    grads = [torch.empty(p["prob"].ffd_shape, dtype=torch.float32, device="cuda") for p in problems]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                               # warm-up outside capture
        batch.grad(inputs, vals, grads)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.grad(inputs, vals, grads)
    for rep, scale in enumerate([1.0, 0.5, -0.75]):
        for (f, m, d), p in zip(inputs, problems):
            d.copy_(p["ffd"] * scale)
        graph.replay()
        torch.cuda.synchronize()
        got_v = vals.clone()
        got_g = [g.clone() for g in grads]
        ref_v, ref_g = batch.grad(inputs)                       # eager, between replays
        torch.cuda.synchronize()
        for i in range(len(problems)):
            assert abs(float(got_v[i]) - float(ref_v[i])) <= 1e-12 * abs(float(ref_v[i])), (rep, i)
            assert rel(got_g[i].cpu().numpy(), ref_g[i].cpu().numpy()) <= 1e-6, (rep, i)
        print(f"replay {rep}: D[0]={float(got_v[0]):.12f}", flush=True)


def test_batched_rejects_mixed_roles_and_short_workspace(problems):
    import ctypes
    import paper_1804_05061_amd as S
    from paper_1804_05061_amd import _lib
    p0 = problems[0]["prob"]
    other = S.Plan(S.Problem(p0.fixed_dims, p0.moving_dims, NB, K, DELTA, S.MOVING_AS_B))
    with pytest.raises(S.SrwcrError, match="INVALID_ARG"):
        S.Batch([problems[0]["plan"], other])
    with pytest.raises(ValueError):
        S.Batch([])
    batch = S.Batch([problems[0]["plan"]])
    items = (_lib.SrwcrBatchItem * 1)()
    v = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty(p0.ffd_shape, dtype=torch.float32, device="cuda")
    p = problems[0]
    items[0] = _lib.SrwcrBatchItem(p["f"].data_ptr(), p["m"].data_ptr(), p["ffd"].data_ptr(), v.data_ptr(),
                                   g.data_ptr())
    L = _lib.load()
    rc = L.srwcr_grad_batched(batch._h, items, ctypes.c_void_p(batch.workspace.data_ptr()),
                              batch.workspace_bytes - 1, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -3                                             # SRWCR_E_WORKSPACE


@pytest.mark.timeout(900)
def test_breathing4d_full_size(orc):
    """Workload 5 as `bench.py --workload breathing4d` times it: 9 phase pairs
    of a 256x256x{80..128} CT-like phantom x 3 pyramid levels = 27 problems
    (69,976,064 voxels), 64 bins, 6x6x6 spatial bins, FFD spacing 10, one
    batched call.  FP32: every problem against the FP64 oracle (value 1e-5,
    gradient 1e-4).  BF16 storage: every third problem against the oracle on
    the stored values (arithmetic only, same gates)."""
    import os

    import paper_1804_05061_amd as S
    nb, Kb, db = 64, (6, 6, 6), (10, 10, 10)
    pairs = synth.breathing_phases(workers=min(8, os.cpu_count() or 1), mp_context="spawn")
    print(f"generated {len(pairs)} phase pairs", flush=True)
    probs = []
    for pi, (f_raw, m_raw) in enumerate(pairs):
        fg = S.normalize(torch.from_numpy(f_raw).cuda(), f_raw.min(), f_raw.max(), nb).cpu().numpy()
        mg = S.normalize(torch.from_numpy(m_raw).cuda(), m_raw.min(), m_raw.max(), nb).cpu().numpy()
        fo = orc.normalize(f_raw, f_raw.min(), f_raw.max(), nb)
        mo = orc.normalize(m_raw, m_raw.min(), m_raw.max(), nb)
        assert np.array_equal(fg, fo) and np.array_equal(mg, mo)
        for lv, (f_l, m_l) in enumerate(zip(synth.pyramid(fo), synth.pyramid(mo))):
            nz, ny, nx = f_l.shape
            probs.append(dict(dims=(nx, ny, nz), f=f_l, m=m_l, pair=pi, level=lv))
    assert sum(int(np.prod(p["dims"])) for p in probs) == 69976064
    for dtype, tdt, every in ((S.F32, torch.float32, 1), (S.BF16, torch.bfloat16, 3)):
        plans, inputs, ffds = [], [], []
        for p in probs:
            prob = S.Problem(p["dims"], p["dims"], nb, Kb, db, S.MOVING_AS_A, dtype, dtype)
            ffd = synth.breathing4d_ffd(prob.ctrl_dims, p["pair"], p["level"])
            plans.append(S.Plan(prob))
            inputs.append((torch.from_numpy(p["f"]).cuda().to(tdt), torch.from_numpy(p["m"]).cuda().to(tdt),
                           torch.from_numpy(ffd).cuda()))
            ffds.append(ffd)
        vals, grads = S.Batch(plans).grad(inputs)
        torch.cuda.synchronize()
        worst_v = worst_g = 0.0
        for i, p in enumerate(probs):
            if i % every:
                continue
            P = orc.Problem(p["dims"], p["dims"], nb, Kb, db, 0)
            f_st, m_st = (inputs[i][0].float().cpu().numpy(), inputs[i][1].float().cpu().numpy())
            Dr, gr = orc.gradient(P, f_st, m_st, ffds[i])
            Db, gb = float(vals[i]), grads[i].cpu().numpy().astype(np.float64)
            ev, eg = abs(Db - Dr) / abs(Dr), rel(gb, gr)
            worst_v, worst_g = max(worst_v, ev), max(worst_g, eg)
            assert ev <= 1e-5 and eg <= 1e-4, (dtype, i, p["dims"], ev, eg)
        print(f"breathing4d dtype={dtype}: worst value rel {worst_v:.2e}, worst gradient rel L2 {worst_g:.2e}",
              flush=True)
        del plans, inputs, vals, grads
