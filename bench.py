"""Benchmark: SRWCR value+gradient voxel-evaluations per second at 256x256x128.

One step = one srwcr_grad call on the CT-like 256x256x128 FP32 workload
(64 intensity bins, 6x6x6 spatial bins, FFD spacing 10, moving image as A,
displacements N(0, 2 vox)): the FFD warp, the joint-moment value pass, the FP64
finalisation and the gradient pass with its scatter to the control points.
Inputs are resident in device memory before the timed region starts.

Prints ONE JSON line.  `roofline` covers the dominant kernel: algorithmic
bytes (the fixed and moving volumes read once per pass) over its mean
duration, timed with HIP events recorded on the launch stream.  `cpu_baseline`
times the FP64 CPU oracle on a bounded z-slab of the same workload.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-slices", type=int, default=32, help="z-slices of the oracle sample")
    ap.add_argument("--cold", action="store_true", help="also time steps with the last-level cache flushed")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"])
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path has no multi-GPU mode",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1804_05061_amd as S
    from workloads import synth

    torch.cuda.set_device(0)
    t0 = time.time()
    w = synth.ct_phantom()
    nb, K, delta = w.n_bins, w.spatial_bins, w.ctrl_spacing
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
    ffd_np = synth.random_ffd(prob.ctrl_dims, 2.0, 2)
    ffd = torch.from_numpy(ffd_np).cuda()
    plan = S.Plan(prob)
    vbuf = torch.empty((), dtype=torch.float64, device="cuda")
    gbuf = torch.empty(prob.ffd_shape, dtype=torch.float32, device="cuda")
    nvox = int(np.prod(w.fixed_dims))

    for _ in range(args.warmup):
        plan.grad(f, m, ffd, vbuf, gbuf)
    torch.cuda.synchronize()
    print(f"[bench] warm-up done ({args.warmup} steps), plan {plan.info()}", file=sys.stderr, flush=True)

    plan.profile(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        plan.grad(f, m, ffd, vbuf, gbuf)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = plan.profile_read()
    plan.profile(False)
    ms_step = 1e3 * elapsed / args.steps
    D = float(vbuf.item())
    print(f"[bench] {args.steps} steps in {elapsed:.4f}s, D={D:.10f}, phases(ms total)={prof}", file=sys.stderr,
          flush=True)

    # dominant kernel and its roofline (algorithmic bytes: F and M read once per pass)
    bytes_f = {"f32": 4, "f16": 2, "bf16": 2}[args.dtype]
    alg_bytes = bytes_f * (nvox + int(np.prod(w.moving_dims)))
    kern = {"srwcr_value_pass": prof["value"] / prof["calls"], "srwcr_grad_pass": prof["grad"] / prof["calls"]}
    dom = max(kern, key=kern.get)
    achieved = alg_bytes / (kern[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "alg_bytes_per_launch": alg_bytes, "mean_ms": round(kern[dom], 5),
                "phase_ms": {k: round(v / prof["calls"], 5) for k, v in prof.items() if k != "calls"}}

    cold = None
    if args.cold:
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

    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        nz = min(args.cpu_slices, w.fixed.shape[0])
        fo = O.normalize(w.fixed, flo, fhi, nb)
        mo = O.normalize(w.moving, mlo, mhi, nb)
        fz, mz = np.ascontiguousarray(fo[:nz]), np.ascontiguousarray(mo[:nz])
        Pz = O.Problem((w.fixed_dims[0], w.fixed_dims[1], nz), (w.moving_dims[0], w.moving_dims[1], nz), nb, K,
                       delta, 0)
        ffd_z = synth.random_ffd(Pz.ctrl_dims, 2.0, 2)
        a = time.perf_counter()
        O.gradient(Pz, fz, mz, ffd_z)
        dt_cpu = time.perf_counter() - a
        vox = w.fixed_dims[0] * w.fixed_dims[1] * nz
        cpu = {"value": round(vox / dt_cpu, 1), "unit": "voxel-evals/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"value+gradient of z-slices 0..{nz - 1} ({vox} voxels) of the same workload, 1 run, "
                         f"{dt_cpu:.2f}s"}

    value = nvox / (ms_step * 1e-3)
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "voxel-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dt[2], "data": "synthetic",
        "config": {"workload": f"{w.name} CT-like phantom, {dt[2]} storage, {nb} bins, {K[0]}x{K[1]}x{K[2]} "
                               f"spatial bins, FFD spacing {delta[0]}, moving as A, Phi~N(0,2 vox)",
                   "voxels": nvox, "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "D": D,
    }
    if cold is not None:
        line["cold_ms_per_step"] = round(cold, 5)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
