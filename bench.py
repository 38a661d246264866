"""Benchmark: SRWCR value+gradient voxel-evaluations per second at 256x256x128.

One step = one srwcr_grad call on the CT-like 256x256x128 FP32 workload
(64 intensity bins, 6x6x6 spatial bins, FFD spacing 10, moving image as A,
displacements N(0, 2 vox)): the FFD warp, the joint-moment value pass, the FP64
finalisation and the gradient pass with its scatter to the control points.
Inputs are resident in device memory before the timed region starts.

Prints ONE JSON line.  `roofline` covers the dominant kernel (the value
pass on the 6x6x6-bin workload, the gradient pass with the regions at the
FFD nodes), named by 10 steps with every phase recorded before the timed
ones: algorithmic bytes (the fixed and moving volumes read once) over its
mean duration, timed with one HIP event pair per timed step recorded on the
launch stream around that pass.  `cold_ms_per_step` is the median of 10 more
steps with the last-level cache flushed before each.  `cpu_baseline`
times the FP64 CPU oracle on the whole workload with all host threads (and on
one core over a z-slab); the same oracle run certifies the measured step:
`parity` holds the value's relative error and the gradient's relative L2
error against it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SRWCR value+gradient voxel-evals/s at 256x256x128; % of HBM roofline"
KERNEL_SOURCE = os.path.join(ROOT, "paper_1804_05061_amd", "csrc", "srwcr_kernels.hip")

# HBM traffic of the dominant kernel per launch, from rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE) over this benchmark, each scaled by what the
# same counter reads for k_normalize, a copy of known size (32 MiB read,
# 32 MiB written at 256x256x128 FP32): fetch x 2.00, write x 1.00.  Keyed by
# the SHA-256 of the kernel source the counters were taken on and by the
# workload, so the figure is reported as null once the kernels change.
TRAFFIC = {
    ("fe2cf65d0b19dba09e481f0468d546a4cbabd22e8882eaed58a9f481dffb162c", "ct256", "srwcr_value_pass", "f32"): {
        "fetch_bytes": 100904234, "write_bytes": 33300480, "fetch_size_kib": 49307.7, "write_size_kib": 32520.0,
        "scale_fetch": 1.9985, "scale_write": 1.0, "copy_kernel": "k_normalize, 32 MiB in, 32 MiB out"},
}

# Issue counters of the same kernel, from rocprofv3's derived metrics over
# SQ_ACTIVE_INST_VALU, SQ_LDS_BANK_CONFLICT and GRBM_GUI_ACTIVE (one XCD's
# cycles), with the same key.  `limiter` names what bounds the kernel: the
# value pass is bound by vector instruction issue (its lane instructions per
# voxel are SQ_INSTS_VALU x 64 / voxels), not by HBM.
ISSUE = {
    ("fe2cf65d0b19dba09e481f0468d546a4cbabd22e8882eaed58a9f481dffb162c", "ct256", "srwcr_value_pass", "f32"): {
        "VALUBusy": 0.6937, "LDSBankConflict": 0.0234, "valu_insts": 93091136, "lds_insts": 3782578,
        "lane_insts_per_voxel": 710.2, "limiter": "valu-issue"},
}


def kernel_source_sha():
    import hashlib
    with open(KERNEL_SOURCE, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-slices", type=int, default=8, help="z-slices of the one-core oracle sample")
    ap.add_argument("--no-cold", action="store_true",
                    help="skip the 10 extra steps timed with the last-level cache flushed before each")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--workload", default="ct256", choices=["ct256", "nodes256x99", "breathing4d", "raptor256"],
                    help="ct256: the headline single pair; nodes256x99: the paper's own setting (regions at the "
                         "FFD nodes, delta 5, 32 bins) on a 256x256x99 phantom; breathing4d: 9 phase pairs x 3 "
                         "levels, batched; raptor256: RaPTOR value+gradient over 17^3 patches of the ct256 pair")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path has no multi-GPU mode",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "breathing4d":
        return bench_breathing4d(args)
    if args.workload == "raptor256":
        return bench_raptor256(args)
    import numpy as np
    import torch

    import paper_1804_05061_amd as S
    from workloads import synth

    torch.cuda.set_device(0)
    t0 = time.time()
    nodes = args.workload == "nodes256x99"
    if nodes:
        # the paper's operating point: regions at the control points, delta 5, 32 bins, 256x256x99
        w = synth.ct_phantom(shape=(99, 256, 256))
        nb, K, delta, phi_sigma, phi_seed = 32, (0, 0, 0), (5, 5, 5), 1.5, 51
    else:
        w = synth.ct_phantom()
        nb, K, delta, phi_sigma, phi_seed = w.n_bins, w.spatial_bins, w.ctrl_spacing, 2.0, 2
    print(f"[bench] workload {w.name} generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    dt = {"f32": (S.F32, torch.float32, "f32"), "f16": (S.F16, torch.float16, "f16"),
          "bf16": (S.BF16, torch.bfloat16, "bf16")}[args.dtype]
    prob = S.Problem(w.fixed_dims, w.moving_dims, nb, K, delta, S.MOVING_AS_A, dt[0], dt[0])
    fr = torch.from_numpy(w.fixed).cuda()
    mr = torch.from_numpy(w.moving).cuda()
    flo, fhi = S.minmax(fr)
    mlo, mhi = S.minmax(mr)
    f = S.normalize(fr, flo, fhi, nb, dt[1])
    m = S.normalize(mr, mlo, mhi, nb, dt[1])
    ffd_np = synth.random_ffd(prob.ctrl_dims, phi_sigma, phi_seed)
    ffd = torch.from_numpy(ffd_np).cuda()
    plan = S.Plan(prob)
    vbuf = torch.empty((), dtype=torch.float64, device="cuda")
    gbuf = torch.empty(prob.ffd_shape, dtype=torch.float32, device="cuda")
    nvox = int(np.prod(w.fixed_dims))

    for _ in range(args.warmup):
        plan.grad(f, m, ffd, vbuf, gbuf)
    torch.cuda.synchronize()
    print(f"[bench] warm-up done ({args.warmup} steps), plan {plan.info()}", file=sys.stderr, flush=True)

    # 10 steps with every phase recorded give the breakdown and name the
    # dominant pass (value or gradient); the timed steps then record one HIP
    # event pair per call, around that pass only (events between all kernels
    # would slow the steps)
    plan.profile(1)
    for _ in range(10):
        plan.grad(f, m, ffd, vbuf, gbuf)
    prof = plan.profile_read()
    dom_phase = "value" if prof["value"] >= prof["grad"] else "grad"
    dom = {"value": "srwcr_value_pass", "grad": "srwcr_gradient_pass"}[dom_phase]
    plan.profile(2 if dom_phase == "value" else 3)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        plan.grad(f, m, ffd, vbuf, gbuf)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof_d = plan.profile_read()
    plan.profile(0)
    ms_step = 1e3 * elapsed / args.steps
    D = float(vbuf.item())
    print(f"[bench] {args.steps} steps in {elapsed:.4f}s, D={D:.10f}, {dom} {prof_d[dom_phase]:.4f} ms total, "
          f"phases of 10 earlier steps (ms total)={prof}", file=sys.stderr, flush=True)

    # dominant kernel and its roofline (algorithmic bytes: both passes read F
    # and the warped M once, b_F + 4 B per fixed voxel)
    bytes_f = {"f32": 4, "f16": 2, "bf16": 2}[args.dtype]
    alg_bytes = bytes_f * (nvox + int(np.prod(w.moving_dims)))
    mean_ms = prof_d[dom_phase] / prof_d["calls"]
    achieved = alg_bytes / (mean_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "alg_bytes_per_launch": alg_bytes, "mean_ms": round(mean_ms, 5),
                "phase_ms": {k: round(v / prof["calls"], 5) for k, v in prof.items() if k != "calls"}}

    key = (kernel_source_sha(), args.workload, dom, dt[2])
    rec = TRAFFIC.get(key)
    if rec is not None:
        roofline["traffic"] = rec["fetch_bytes"] + rec["write_bytes"]
        roofline["traffic_detail"] = rec
    roofline["issue"] = ISSUE.get(key)
    roofline["limiter"] = roofline["issue"]["limiter"] if roofline["issue"] else None

    cold = None
    if not args.no_cold:
        flush = torch.empty(1 << 29, dtype=torch.uint8, device="cuda")   # 512 MiB > last-level cache
        times = []
        for _ in range(10):
            flush.fill_(1)
            torch.cuda.synchronize()
            a = time.perf_counter()
            plan.grad(f, m, ffd, vbuf, gbuf)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - a)
        cold = 1e3 * float(np.median(times))
        del flush

    # whole step against the same roofline: F and M read once by each of the two passes
    step_bytes = 2 * alg_bytes
    roofline["step"] = {"alg_bytes": step_bytes, "ms": round(ms_step, 5),
                        "achieved": round(step_bytes / (ms_step * 1e-3) / 1e9, 2),
                        "frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 5)}

    cpu, parity = None, None
    if not args.no_cpu:
        g_gpu = gbuf.cpu().numpy().astype(np.float64)
        from oracle import oracle as O
        fo = O.normalize(w.fixed, flo, fhi, nb)
        mo = O.normalize(w.moving, mlo, mhi, nb)
        if args.dtype != "f32":
            # the oracle sees the values as stored (arithmetic-only error), rounded on the host
            fo = torch.from_numpy(fo).to(dt[1]).float().numpy()
            mo = torch.from_numpy(mo).to(dt[1]).float().numpy()
        # the measured configuration through the FP64 oracle on all host threads: the
        # parity of this very step and the all-core baseline
        Po = O.Problem(w.fixed_dims, w.moving_dims, nb, K, delta, 0)
        a = time.perf_counter()
        Dr, gr = O.gradient(Po, fo, mo, ffd_np)
        dt_all = time.perf_counter() - a
        threads = O.num_threads()
        parity = {"value_rel": float(f"{abs(D - Dr) / abs(Dr):.3e}"),
                  "grad_rel_l2": float(f"{np.linalg.norm(g_gpu - gr) / np.linalg.norm(gr):.3e}"),
                  "oracle": "FP64 oracle, same inputs" + (" as stored" if args.dtype != "f32" else "")}
        cpu = {"value": round(nvox / dt_all, 1), "unit": "voxel-evals/s", "cores": threads, "kind": "oracle",
               "sample": f"the whole workload (value+gradient, {nvox} voxels), 1 run, {dt_all:.2f}s"}
        # one core, on a z-slab of the same workload
        nz = min(args.cpu_slices, w.fixed.shape[0])
        fz, mz = np.ascontiguousarray(fo[:nz]), np.ascontiguousarray(mo[:nz])
        Pz = O.Problem((w.fixed_dims[0], w.fixed_dims[1], nz), (w.moving_dims[0], w.moving_dims[1], nz), nb, K,
                       delta, 0)
        ffd_z = synth.random_ffd(Pz.ctrl_dims, phi_sigma, phi_seed)
        O.set_num_threads(1)
        a = time.perf_counter()
        O.gradient(Pz, fz, mz, ffd_z)
        dt_one = time.perf_counter() - a
        O.set_num_threads(threads)
        vox = w.fixed_dims[0] * w.fixed_dims[1] * nz
        cpu["one_core"] = {"value": round(vox / dt_one, 1), "cores": 1,
                           "sample": f"value+gradient of z-slices 0..{nz - 1} ({vox} voxels), 1 run, {dt_one:.2f}s"}

    value = nvox / (ms_step * 1e-3)
    vs = None
    if nodes:
        metric = "SRWCR value+gradient voxel-evals/s at 256x256x99, regions at the FFD nodes"
        regions = f"regions at the FFD nodes ({prob.n_regions} regions)"
        # the paper's own figure for this setting and size: 851 ms (value) + 238 ms
        # (derivatives) per iteration on a GTX 1060 (Table VIII); another machine,
        # context only
        vs = round(value / (nvox / 1.089), 2)
    else:
        metric = METRIC
        regions = f"{K[0]}x{K[1]}x{K[2]} spatial bins"
    line = {
        "metric": metric, "value": round(value, 1), "unit": "voxel-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": vs, "dtype": dt[2], "data": "synthetic",
        "config": {"workload": f"{w.name} CT-like phantom, {dt[2]} storage, {nb} bins, {regions}, "
                               f"FFD spacing {delta[0]}, moving as A, Phi~N(0,{phi_sigma} vox)",
                   "voxels": nvox, "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "D": D, "parity": parity,
    }
    if cold is not None:
        line["cold_ms_per_step"] = round(cold, 5)
    print(json.dumps(line), flush=True)


def bench_breathing4d(args):
    """9 breathing-phase pairs (80..128 of 128 slices of a 256x256 CT-like
    phantom) x 3 pyramid levels = 27 problems, 64 bins, 6x6x6 spatial bins, FFD
    spacing 10 level voxels: one srwcr_grad_batched call (replayed from a HIP
    graph) against 27 plain srwcr_grad calls."""
    import numpy as np

    from workloads import synth
    t0 = time.time()
    pairs = synth.breathing_phases(workers=min(10, os.cpu_count() or 1))    # before the GPU is touched
    print(f"[bench] 9 phase pairs generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    import torch

    import paper_1804_05061_amd as S
    torch.cuda.set_device(0)
    dt = {"f32": (S.F32, torch.float32, 4), "f16": (S.F16, torch.float16, 2),
          "bf16": (S.BF16, torch.bfloat16, 2)}[args.dtype]
    nb, K, delta = 64, (6, 6, 6), (10, 10, 10)
    plans, inputs, alg_bytes, nvox = [], [], 0, 0
    for pi, (f_raw, m_raw) in enumerate(pairs):
        # normalise once at the finest level, then Gaussian (sigma 1 voxel) and every second voxel
        lv_f = synth.pyramid(S.normalize(torch.from_numpy(f_raw).cuda(), f_raw.min(), f_raw.max(), nb).cpu().numpy())
        lv_m = synth.pyramid(S.normalize(torch.from_numpy(m_raw).cuda(), m_raw.min(), m_raw.max(), nb).cpu().numpy())
        for lv in range(3):
            nz, ny, nx = lv_f[lv].shape
            prob = S.Problem((nx, ny, nz), (nx, ny, nz), nb, K, delta, S.MOVING_AS_A, dt[0], dt[0])
            ffd = torch.from_numpy(synth.breathing4d_ffd(prob.ctrl_dims, pi, lv)).cuda()
            plans.append(S.Plan(prob))
            inputs.append((torch.from_numpy(lv_f[lv]).cuda().to(dt[1]), torch.from_numpy(lv_m[lv]).cuda().to(dt[1]),
                           ffd))
            nvox += nx * ny * nz
            alg_bytes += 2 * 2 * dt[2] * nx * ny * nz          # F and M read once per pass, two passes
    batch = S.Batch(plans)
    vals = torch.empty(len(plans), dtype=torch.float64, device="cuda")
    grads = [torch.empty(p.problem.ffd_shape, dtype=torch.float32, device="cuda") for p in plans]
    single_v = [torch.empty((), dtype=torch.float64, device="cuda") for _ in plans]

    def sequential():
        for p, (f, m, d), v, g in zip(plans, inputs, single_v, grads):
            p.grad(f, m, d, v, g)

    def timed(fn, steps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - a) / steps

    for _ in range(args.warmup):
        sequential()
        batch.grad(inputs, vals, grads)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        batch.grad(inputs, vals, grads)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.grad(inputs, vals, grads)
    graph.replay()
    torch.cuda.synchronize()
    ms_seq = timed(sequential, args.steps)
    ms_batch = timed(lambda: batch.grad(inputs, vals, grads), args.steps)
    ms_graph = timed(graph.replay, args.steps)
    D0 = float(vals[0].item())
    print(f"[bench] sequential {ms_seq:.3f} ms, batched {ms_batch:.3f} ms, graph {ms_graph:.3f} ms, D[0]={D0:.10f}",
          file=sys.stderr, flush=True)
    line = {
        "metric": "breathing 4-D batch: SRWCR value+gradient voxel-evals/s (27 problems per evaluation)",
        "value": round(nvox / (ms_graph * 1e-3), 1), "unit": "voxel-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_graph, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"9 breathing-phase pairs x 3 levels of a 256x256x128 CT-like phantom, {args.dtype} "
                               f"storage, {nb} bins, 6x6x6 spatial bins, FFD spacing 10, moving as A",
                   "problems": len(plans), "voxels": nvox, "parallelism": "single GPU"},
        "pairs_per_s": round(len(pairs) / (ms_graph * 1e-3), 2),
        "alg_gb_per_s": round(alg_bytes / (ms_graph * 1e-3) / 1e9, 2),
        "ms_sequential_27_calls": round(ms_seq, 5), "ms_batched_eager": round(ms_batch, 5),
        "ms_batched_graph": round(ms_graph, 5), "speedup_vs_sequential": round(ms_seq / ms_graph, 3),
    }
    print(json.dumps(line), flush=True)


def bench_raptor256(args):
    """RaPTOR (eqs 6, 13, 14) value+gradient on the ct256 pair: 1709 random 17^3
    patches (about one cover of the grid); FFD spacing 10, displacements
    N(0, 1.5 vox), moving as A."""
    import numpy as np
    import torch

    import paper_1804_05061_amd as S
    from workloads import synth

    torch.cuda.set_device(0)
    t0 = time.time()
    w = synth.ct_phantom()
    nb, K, delta = w.n_bins, w.spatial_bins, w.ctrl_spacing
    print(f"[bench] workload {w.name} generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    prob = S.Problem(w.fixed_dims, w.moving_dims, nb, K, delta, S.MOVING_AS_A)
    fr = torch.from_numpy(w.fixed).cuda()
    mr = torch.from_numpy(w.moving).cuda()
    flo, fhi = S.minmax(fr)
    mlo, mhi = S.minmax(mr)
    f = S.normalize(fr, flo, fhi, nb)
    m = S.normalize(mr, mlo, mhi, nb)
    ffd_np = synth.random_ffd(prob.ctrl_dims, 1.5, 43)
    ffd = torch.from_numpy(ffd_np).cuda()
    boxes = synth.raptor_patches(w.fixed_dims, side=17, coverage=1.0, k=44, extra_edge=False)
    plan = S.Plan(prob)
    rp = S.RaptorPatches(plan, boxes)
    vbuf = torch.empty((), dtype=torch.float64, device="cuda")
    gbuf = torch.empty(prob.ffd_shape, dtype=torch.float32, device="cuda")
    nvox = int(np.prod(w.fixed_dims))
    lo = np.maximum(boxes[:, :3], 0)
    hi = np.minimum(boxes[:, 3:], np.array(w.fixed_dims))
    patch_vox = int(np.prod(np.maximum(hi - lo, 0), axis=1).sum())

    for _ in range(args.warmup):
        rp.grad(f, m, ffd, value_out=vbuf, grad_out=gbuf)
    torch.cuda.synchronize()
    # one event pair per timed call around the patch sums, then 10 more calls
    # with every phase recorded for the breakdown
    plan.profile(2)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        rp.grad(f, m, ffd, value_out=vbuf, grad_out=gbuf)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof_v = rp.profile_read()
    plan.profile(1)
    for _ in range(10):
        rp.grad(f, m, ffd, value_out=vbuf, grad_out=gbuf)
    prof = rp.profile_read()
    plan.profile(0)
    ms_step = 1e3 * elapsed / args.steps
    R = float(vbuf.item())
    print(f"[bench] {args.steps} steps in {elapsed:.4f}s, RaPTOR={R:.10f}, patch sums {prof_v['patch_sums']:.4f} ms "
          f"total, phases of 10 more calls (ms total)={prof}", file=sys.stderr, flush=True)

    # algorithmic bytes per launch of each kernel (its inputs read once, its outputs written once):
    #   warp pass: M read once (4 B / moving voxel)
    #   patch sums: the warped sample (8 B) and F (4 B) per patch voxel
    #   derivative: the same 12 B plus the 4 B per-voxel sum per patch voxel
    #   chain rule: the per-voxel sum (4 B) and dM/dy (12 B) per fixed voxel
    alg = {"warp": 4 * int(np.prod(w.moving_dims)), "patch_sums": 12 * patch_vox, "derivative": 16 * patch_vox,
           "chain_rule": 16 * nvox}
    dom = "patch_sums"
    kern = {dom: prof_v[dom] / prof_v["calls"]}
    achieved = alg[dom] / (kern[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None, "alg_bytes_per_launch": alg[dom],
                "mean_ms": round(kern[dom], 5),
                "phase_ms": {k: round(v / prof["calls"], 5) for k, v in prof.items() if k != "calls"}}

    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        fo = O.normalize(w.fixed, flo, fhi, nb)
        mo = O.normalize(w.moving, mlo, mhi, nb)
        Po = O.Problem(w.fixed_dims, w.moving_dims, nb, K, delta, 0)
        a = time.perf_counter()
        O.raptor(Po, fo, mo, ffd_np, boxes, want_grad=True)
        dt_cpu = time.perf_counter() - a
        cpu = {"value": round(nvox / dt_cpu, 1), "unit": "voxel-evals/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"the whole workload (value+gradient, {len(boxes)} patches), 1 run, {dt_cpu:.2f}s"}

    line = {
        "metric": "RaPTOR value+gradient voxel-evals/s at 256x256x128", "value": round(nvox / (ms_step * 1e-3), 1),
        "unit": "voxel-evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{w.name} CT-like phantom, f32 storage, {nb} bins, {len(boxes)} random 17^3 patches "
                               f"({patch_vox} patch voxels), FFD spacing {delta[0]}, moving as A, Phi~N(0,1.5 vox)",
                   "voxels": nvox, "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "RaPTOR": R,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
