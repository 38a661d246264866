"""SRWCR on MI355X: the spatially region-weighted correlation ratio and its
analytic gradient with respect to cubic B-spline FFD displacements
(Gong et al., arXiv 1804.05061), computed by hand-written gfx950 kernels
behind the C ABI of include/srwcr.h.

This module only marshals arguments: PyTorch provides device memory and the
current stream; every step of the computation runs in libsrwcr.so.  Volumes
are torch tensors shaped (nz, ny, nx) on the GPU; FFD displacements are
float32 tensors shaped (3, ncz, ncy, ncx) in fixed-voxel units.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import SrwcrError

MOVING_AS_A, MOVING_AS_B = 0, 1
F32, F16, BF16 = 0, 1, 2
_TORCH_DT = {F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16}
_DT_OF = {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}

__all__ = ["Problem", "Plan", "Batch", "normalize", "minmax", "register_lbfgs", "LbfgsOptions", "SrwcrError",
           "MOVING_AS_A", "MOVING_AS_B", "F32", "F16", "BF16", "SRWCRLoss", "SRWCRDenseLoss", "RaptorPatches",
           "tune"]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _need_cuda(t: torch.Tensor, name: str, dtype=None, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


@dataclass(frozen=True)
class Problem:
    """Problem statement (Sec. II): grids (x, y, z), L_eps + 1 intensity bins,
    spatial bins per axis, FFD control spacing, role of the moving image and
    storage dtypes of the normalised volumes."""
    fixed_dims: tuple
    moving_dims: tuple
    n_bins: int
    spatial_bins: tuple
    ctrl_spacing: tuple
    role: int = MOVING_AS_A
    fixed_dtype: int = F32
    moving_dtype: int = F32

    def c(self) -> _lib.SrwcrProblem:
        p = _lib.SrwcrProblem()
        p.fixed_dims[:] = [int(v) for v in self.fixed_dims]
        p.moving_dims[:] = [int(v) for v in self.moving_dims]
        p.n_bins = int(self.n_bins)
        p.spatial_bins[:] = [int(v) for v in self.spatial_bins]
        p.ctrl_spacing[:] = [int(v) for v in self.ctrl_spacing]
        p.role = int(self.role)
        p.fixed_dtype = int(self.fixed_dtype)
        p.moving_dtype = int(self.moving_dtype)
        return p

    @property
    def ctrl_dims(self) -> tuple:
        nc = (ctypes.c_int32 * 3)()
        _lib.check(_lib.load().srwcr_ctrl_dims(ctypes.byref(self.c()), nc))
        return tuple(nc)

    @property
    def fixed_shape(self):
        return tuple(self.fixed_dims[::-1])

    @property
    def moving_shape(self):
        return tuple(self.moving_dims[::-1])

    @property
    def ffd_shape(self):
        return (3,) + tuple(self.ctrl_dims[::-1])

    @property
    def field_shape(self):
        """Dense displacement field u[3][nz][ny][nx] on the fixed grid."""
        return (3,) + tuple(self.fixed_dims[::-1])

    @property
    def at_nodes(self) -> bool:
        """spatial_bins (0, 0, 0): the regions are the FFD nodes (Sec. II-C)."""
        return tuple(self.spatial_bins) == (0, 0, 0)

    @property
    def n_regions(self) -> int:
        k = self.ctrl_dims if self.at_nodes else self.spatial_bins
        return int(k[0]) * int(k[1]) * int(k[2])


class Plan:
    """A plan (device tables and launch geometry) plus its own workspace."""

    def __init__(self, problem: Problem, device=None, tuning=None):
        """tuning: None, or a dict with grad_item_voxels / value_workgroups
        (see `tune`; 0 or missing keeps the default)."""
        self.problem = problem
        self.tuning = dict(tuning or {})
        L = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        with torch.cuda.device(self.device):
            h = ctypes.c_void_p()
            t = _lib.SrwcrTuning(int(self.tuning.get("grad_item_voxels", 0)),
                                 int(self.tuning.get("value_workgroups", 0)))
            _lib.check(L.srwcr_plan_create_tuned(ctypes.byref(problem.c()), ctypes.byref(t), ctypes.byref(h)))
            self._h = h
            self.workspace_bytes = int(L.srwcr_workspace_bytes(h))
            self.workspace = torch.zeros(self.workspace_bytes, dtype=torch.uint8, device=self.device)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.load().srwcr_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        n, v, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.load().srwcr_plan_info(self._h, ctypes.byref(n), ctypes.byref(v), ctypes.byref(g)))
        return {"n_items": n.value, "value_lds": v.value, "grad_lds": g.value}

    def _check_inputs(self, fixed, moving, ffd):
        p = self.problem
        _need_cuda(fixed, "fixed", _TORCH_DT[p.fixed_dtype], p.fixed_shape)
        _need_cuda(moving, "moving", _TORCH_DT[p.moving_dtype], p.moving_shape)
        _need_cuda(ffd, "ffd", torch.float32, p.ffd_shape)

    def eval(self, fixed, moving, ffd, out=None):
        """SRWCR value D (eq 9) as a 0-dim float64 device tensor."""
        self._check_inputs(fixed, moving, ffd)
        if out is None:
            out = torch.empty((), dtype=torch.float64, device=fixed.device)
        _lib.check(_lib.load().srwcr_eval(self._h, _ptr(fixed), _ptr(moving), _ptr(ffd), _ptr(out),
                                          _ptr(self.workspace), self.workspace_bytes, _stream()))
        return out

    def grad(self, fixed, moving, ffd, value_out=None, grad_out=None):
        """(D, dD/d displacement) -- eqs (15)-(21)."""
        self._check_inputs(fixed, moving, ffd)
        if value_out is None:
            value_out = torch.empty((), dtype=torch.float64, device=fixed.device)
        if grad_out is None:
            grad_out = torch.empty(self.problem.ffd_shape, dtype=torch.float32, device=fixed.device)
        _lib.check(_lib.load().srwcr_grad(self._h, _ptr(fixed), _ptr(moving), _ptr(ffd), _ptr(value_out),
                                          _ptr(grad_out), _ptr(self.workspace), self.workspace_bytes, _stream()))
        return value_out, grad_out

    def grad_noalloc(self, fixed, moving, ffd, value_out, grad_out):
        """grad() on the library's static device workspace instead of the plan's
        (srwcr_grad_noalloc); the caller passes both outputs."""
        self._check_inputs(fixed, moving, ffd)
        _need_cuda(value_out, "value_out", torch.float64, ())
        _need_cuda(grad_out, "grad_out", torch.float32, self.problem.ffd_shape)
        _lib.check(_lib.load().srwcr_grad_noalloc(self._h, _ptr(fixed), _ptr(moving), _ptr(ffd), _ptr(value_out),
                                                  _ptr(grad_out), _stream()))
        return value_out, grad_out

    def _check_dense(self, fixed, moving, field):
        p = self.problem
        _need_cuda(fixed, "fixed", _TORCH_DT[p.fixed_dtype], p.fixed_shape)
        _need_cuda(moving, "moving", _TORCH_DT[p.moving_dtype], p.moving_shape)
        _need_cuda(field, "field", torch.float32, p.field_shape)

    def eval_dense(self, fixed, moving, field, out=None):
        """D with the warp T(x) = x + u(x) of a dense field u[3][nz][ny][nx]."""
        self._check_dense(fixed, moving, field)
        if out is None:
            out = torch.empty((), dtype=torch.float64, device=fixed.device)
        _lib.check(_lib.load().srwcr_eval_dense(self._h, _ptr(fixed), _ptr(moving), _ptr(field), _ptr(out),
                                                _ptr(self.workspace), self.workspace_bytes, _stream()))
        return out

    def grad_dense(self, fixed, moving, field, value_out=None, grad_out=None):
        """(D, dD/du[3][nz][ny][nx]) for a dense displacement field (eq 16 per voxel)."""
        self._check_dense(fixed, moving, field)
        if value_out is None:
            value_out = torch.empty((), dtype=torch.float64, device=fixed.device)
        if grad_out is None:
            grad_out = torch.empty(self.problem.field_shape, dtype=torch.float32, device=fixed.device)
        _lib.check(_lib.load().srwcr_grad_dense(self._h, _ptr(fixed), _ptr(moving), _ptr(field), _ptr(value_out),
                                                _ptr(grad_out), _ptr(self.workspace), self.workspace_bytes,
                                                _stream()))
        return value_out, grad_out

    def grad_fixed(self, fixed, moving, disp, dense: bool = False, value_out=None, grad_out=None):
        """(D, dD/ds_F[nz][ny][nx]): the derivative with respect to the normalised
        fixed intensity per voxel; disp is the FFD, or a dense field when dense."""
        if dense:
            self._check_dense(fixed, moving, disp)
        else:
            self._check_inputs(fixed, moving, disp)
        if value_out is None:
            value_out = torch.empty((), dtype=torch.float64, device=fixed.device)
        if grad_out is None:
            grad_out = torch.empty(self.problem.fixed_shape, dtype=torch.float32, device=fixed.device)
        _need_cuda(grad_out, "grad_out", torch.float32, self.problem.fixed_shape)
        _lib.check(_lib.load().srwcr_grad_fixed(self._h, _ptr(fixed), _ptr(moving), _ptr(disp), 1 if dense else 0,
                                                _ptr(value_out), _ptr(grad_out), _ptr(self.workspace),
                                                self.workspace_bytes, _stream()))
        return value_out, grad_out

    def warp(self, moving, ffd, out=None):
        """Backward-warped moving volume on the fixed grid (float32)."""
        p = self.problem
        _need_cuda(moving, "moving", _TORCH_DT[p.moving_dtype], p.moving_shape)
        _need_cuda(ffd, "ffd", torch.float32, p.ffd_shape)
        if out is None:
            out = torch.empty(p.fixed_shape, dtype=torch.float32, device=moving.device)
        _lib.check(_lib.load().ffd_warp(self._h, _ptr(moving), _ptr(ffd), _ptr(out), _stream()))
        return out

    def profile(self, enable):
        """Start per-kernel HIP-event timing of grad() (True or 1: every phase;
        2: only the value pass, 3: only the gradient pass, one event pair per
        call) or stop it (False, 0)."""
        _lib.check(_lib.load().srwcr_profile(self._h, int(enable)))

    def profile_read(self) -> dict:
        """Summed milliseconds per phase of the grad() calls recorded so far."""
        ms = (ctypes.c_double * 6)()
        n = ctypes.c_int32()
        _lib.check(_lib.load().srwcr_profile_read(self._h, ms, ctypes.byref(n)))
        names = ["zero", "warp", "value", "finalize", "grad", "grad_out"]
        return {"calls": n.value, **{k: ms[i] for i, k in enumerate(names)}}

    def debug_moments(self, fixed, moving, ffd):
        """Raw (P, S1, S2) moment slots [R, n_bins, 3] of the value pass."""
        self._check_inputs(fixed, moving, ffd)
        R = self.problem.n_regions
        out = torch.empty((R, self.problem.n_bins, 3), dtype=torch.float64, device=fixed.device)
        _lib.check(_lib.load().srwcr_debug_moments(self._h, _ptr(fixed), _ptr(moving), _ptr(ffd), _ptr(out),
                                                   _ptr(self.workspace), self.workspace_bytes, _stream()))
        return out


    def debug_samples(self, moving, ffd):
        """Per fixed voxel, the warp pass's moving bin k (int32) and in-bin
        position s - k (float32), shaped like the fixed volume."""
        p = self.problem
        _need_cuda(moving, "moving", _TORCH_DT[p.moving_dtype], p.moving_shape)
        _need_cuda(ffd, "ffd", torch.float32, p.ffd_shape)
        k = torch.empty(p.fixed_shape, dtype=torch.int32, device=moving.device)
        t = torch.empty(p.fixed_shape, dtype=torch.float32, device=moving.device)
        _lib.check(_lib.load().srwcr_debug_samples(self._h, _ptr(moving), _ptr(ffd), _ptr(k), _ptr(t),
                                                   _ptr(self.workspace), self.workspace_bytes, _stream()))
        return k, t

def _tune_key(problem: Problem, device) -> str:
    p = problem
    return (f"{torch.cuda.get_device_name(device)}|{tuple(p.fixed_dims)}|{tuple(p.moving_dims)}|{p.n_bins}|"
            f"{tuple(p.spatial_bins)}|{tuple(p.ctrl_spacing)}|{p.role}|{p.fixed_dtype}|{p.moving_dtype}")


def tune(problem: Problem, fixed, moving, ffd, item_voxels=None, workgroups=None, steps: int = 10,
         cache: str | None = None) -> dict:
    """Autotune a plan's launch shape on the caller's data: every candidate
    (gradient-pass item size x value-pass workgroup count) is timed over
    `steps` srwcr_grad calls after a warm-up, and the fastest is returned as
    {"grad_item_voxels", "value_workgroups", "ms", "timings"}.  Candidates
    default to |F| / (1200, 600, 300) voxels per item and (1/2, 1) x the
    compute units.  With `cache` (a JSON file, default $SRWCR_TUNE_CACHE), a
    result for the same problem and device is reused and new ones are
    stored."""
    import json
    import os
    import time
    cache = cache or os.environ.get("SRWCR_TUNE_CACHE")
    device = fixed.device
    key = _tune_key(problem, device)
    db = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            db = json.load(fh)
        if key in db:
            return db[key]
    nvox = int(problem.fixed_dims[0]) * int(problem.fixed_dims[1]) * int(problem.fixed_dims[2])
    ncu = torch.cuda.get_device_properties(device).multi_processor_count
    item_voxels = item_voxels or sorted({max(2048, min(65536, nvox // d)) for d in (1200, 600, 300)})
    workgroups = workgroups or sorted({max(1, ncu // 2), ncu})
    timings = []
    for iv in item_voxels:
        for wg in workgroups:
            plan = Plan(problem, device.index, {"grad_item_voxels": iv, "value_workgroups": wg})
            v = torch.empty((), dtype=torch.float64, device=device)
            g = torch.empty(problem.ffd_shape, dtype=torch.float32, device=device)
            for _ in range(2):
                plan.grad(fixed, moving, ffd, v, g)
            torch.cuda.synchronize(device)
            t0 = time.perf_counter()
            for _ in range(steps):
                plan.grad(fixed, moving, ffd, v, g)
            torch.cuda.synchronize(device)
            timings.append({"grad_item_voxels": iv, "value_workgroups": wg,
                            "ms": 1e3 * (time.perf_counter() - t0) / steps})
            del plan
    best = dict(min(timings, key=lambda r: r["ms"]))
    best["timings"] = timings
    if cache:
        db[key] = best
        with open(cache, "w") as fh:
            json.dump(db, fh, indent=1)
    return best


class Batch:
    """Independent problems (plans) evaluated by one launch per pass
    (srwcr_grad_batched).  The plans must share role and storage dtypes and
    are kept alive by the batch."""

    def __init__(self, plans):
        plans = list(plans)
        if not 1 <= len(plans) <= _lib.MAX_BATCH:
            raise ValueError(f"a batch holds 1..{_lib.MAX_BATCH} plans, got {len(plans)}")
        self.plans = plans
        self.device = plans[0].device
        L = _lib.load()
        arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
        with torch.cuda.device(self.device):
            h = ctypes.c_void_p()
            _lib.check(L.srwcr_batch_create(len(plans), arr, ctypes.byref(h)))
            self._h = h
            self.workspace_bytes = int(L.srwcr_batch_workspace_bytes(h))
            self.workspace = torch.zeros(self.workspace_bytes, dtype=torch.uint8, device=self.device)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.load().srwcr_batch_destroy(h)
            except Exception:
                pass
            self._h = None

    def grad(self, inputs, values=None, grads=None):
        """inputs: [(fixed, moving, ffd)] per plan.  Returns (values float64
        tensor [n], [dD/d displacement per problem])."""
        n = len(self.plans)
        if len(inputs) != n:
            raise ValueError(f"{len(inputs)} inputs for {n} plans")
        for pl, (f, m, d) in zip(self.plans, inputs):
            pl._check_inputs(f, m, d)
        if values is None:
            values = torch.empty(n, dtype=torch.float64, device=self.device)
        if grads is None:
            grads = [torch.empty(pl.problem.ffd_shape, dtype=torch.float32, device=self.device) for pl in self.plans]
        _need_cuda(values, "values", torch.float64, (n,))
        for pl, g in zip(self.plans, grads):
            _need_cuda(g, "grad", torch.float32, pl.problem.ffd_shape)
        items = (_lib.SrwcrBatchItem * n)()
        for i, ((f, m, d), g) in enumerate(zip(inputs, grads)):
            items[i] = _lib.SrwcrBatchItem(_ptr(f), _ptr(m), _ptr(d), values.data_ptr() + 8 * i, _ptr(g))
        _lib.check(_lib.load().srwcr_grad_batched(self._h, items, _ptr(self.workspace), self.workspace_bytes,
                                                  _stream()))
        return values, grads


class RaptorPatches:
    """RaPTOR (eqs 6, 13, 14) over a fixed set of boxcar patches on a plan:
    `boxes` is an int array [n, 6] of half-open boxes (x0, y0, z0, x1, y1, z1)
    on the fixed grid.  Holds the device patch tables and its own workspace;
    the plan is kept alive by the set."""

    def __init__(self, plan: Plan, boxes):
        import numpy as np
        b = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32).reshape(-1, 6))
        self.plan = plan
        self.n = len(b)
        arr = (_lib.SrwcrPatch * max(self.n, 1))()
        for i, r in enumerate(b.tolist()):
            arr[i] = _lib.SrwcrPatch(*r)
        L = _lib.load()
        with torch.cuda.device(plan.device):
            h = ctypes.c_void_p()
            _lib.check(L.raptor_patches_create(plan.handle, arr, self.n, ctypes.byref(h)))
            self._h = h
            self.workspace_bytes = int(L.raptor_workspace_bytes(plan.handle, h))
            self.workspace = torch.zeros(self.workspace_bytes, dtype=torch.uint8, device=plan.device)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                _lib.load().raptor_patches_destroy(h)
            except Exception:
                pass
            self._h = None

    def _check(self, fixed, moving, disp, dense):
        p = self.plan.problem
        _need_cuda(fixed, "fixed", _TORCH_DT[p.fixed_dtype], p.fixed_shape)
        _need_cuda(moving, "moving", _TORCH_DT[p.moving_dtype], p.moving_shape)
        _need_cuda(disp, "disp", torch.float32, p.field_shape if dense else p.ffd_shape)

    def eval(self, fixed, moving, disp, dense: bool = False, out=None):
        """RaPTOR (eq 13) as a 0-dim float64 device tensor; disp is the FFD, or
        a dense field [3][nz][ny][nx] when dense."""
        self._check(fixed, moving, disp, dense)
        if out is None:
            out = torch.empty((), dtype=torch.float64, device=fixed.device)
        _lib.check(_lib.load().raptor_eval(self.plan.handle, self._h, _ptr(fixed), _ptr(moving), _ptr(disp),
                                           1 if dense else 0, _ptr(out), _ptr(self.workspace),
                                           self.workspace_bytes, _stream()))
        return out

    def profile_read(self) -> dict:
        """Summed milliseconds per phase of the grad() calls recorded since
        plan.profile(True)."""
        ms = (ctypes.c_double * 6)()
        n = ctypes.c_int32()
        _lib.check(_lib.load().srwcr_profile_read(self.plan.handle, ms, ctypes.byref(n)))
        names = ["zero", "warp", "patch_sums", "patch_finalize", "derivative", "chain_rule"]
        return {"calls": n.value, **{k: ms[i] for i, k in enumerate(names)}}

    def grad(self, fixed, moving, disp, dense: bool = False, value_out=None, grad_out=None):
        """(RaPTOR, dRaPTOR/d disp), the gradient shaped like disp."""
        self._check(fixed, moving, disp, dense)
        p = self.plan.problem
        if value_out is None:
            value_out = torch.empty((), dtype=torch.float64, device=fixed.device)
        if grad_out is None:
            grad_out = torch.empty(p.field_shape if dense else p.ffd_shape, dtype=torch.float32, device=fixed.device)
        _lib.check(_lib.load().raptor_grad(self.plan.handle, self._h, _ptr(fixed), _ptr(moving), _ptr(disp),
                                           1 if dense else 0, _ptr(value_out), _ptr(grad_out),
                                           _ptr(self.workspace), self.workspace_bytes, _stream()))
        return value_out, grad_out


def normalize(raw: torch.Tensor, lo: float, hi: float, n_bins: int, dtype=torch.float32) -> torch.Tensor:
    """Intensities mapped linearly to [0, L_eps] (Sec. II), stored in `dtype`."""
    _need_cuda(raw, "raw", torch.float32)
    out = torch.empty(raw.shape, dtype=dtype, device=raw.device)
    _lib.check(_lib.load().srwcr_normalize(_ptr(raw), raw.numel(), float(lo), float(hi), int(n_bins), _ptr(out),
                                           _DT_OF[dtype], _stream()))
    return out


def minmax(raw: torch.Tensor):
    """(min, max) of a float32 device volume; raises on NaN / Inf."""
    _need_cuda(raw, "raw", torch.float32)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    _lib.check(_lib.load().srwcr_minmax(_ptr(raw), raw.numel(), ctypes.byref(lo), ctypes.byref(hi), _stream()))
    return lo.value, hi.value


@dataclass
class LbfgsOptions:
    levels: int = 3
    max_iter: tuple = (200, 200, 120)
    history: int = 5
    stall_window: int = 20
    stall_tol: float = 1e-6
    bending_weight: float = 0.0

    def c(self) -> _lib.SrwcrLbfgsOpts:
        o = _lib.SrwcrLbfgsOpts()
        o.levels = self.levels
        o.max_iter[:] = list(self.max_iter)
        o.history = self.history
        o.stall_window = self.stall_window
        o.stall_tol = self.stall_tol
        o.bending_weight = self.bending_weight
        return o


def register_lbfgs(problem: Problem, fixed: torch.Tensor, moving: torch.Tensor, ffd, options=None):
    """Multi-resolution L-BFGS registration (Sec. II-F).  `ffd` is a host float32
    numpy array (3, ncz, ncy, ncx), updated in place; returns the report."""
    import numpy as np
    _need_cuda(fixed, "fixed", torch.float32, problem.fixed_shape)
    _need_cuda(moving, "moving", torch.float32, problem.moving_shape)
    if not (isinstance(ffd, np.ndarray) and ffd.dtype == np.float32 and ffd.flags.c_contiguous):
        raise TypeError("ffd must be a C-contiguous float32 numpy array")
    opts = (options or LbfgsOptions()).c()
    rep = _lib.SrwcrLbfgsReport()
    _lib.check(_lib.load().register_lbfgs(ctypes.byref(problem.c()), _ptr(fixed), _ptr(moving),
                                          ffd.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts),
                                          ctypes.byref(rep), _stream()))
    return {"iterations": list(rep.iterations), "evaluations": list(rep.evaluations),
            "initial_value": list(rep.initial_value), "final_value": list(rep.final_value),
            "status": list(rep.status), "seconds": list(rep.seconds)}


def _fixed_grad(ctx, disp, fixed, moving, dense, grad_output):
    """dD/d(normalised fixed) for a float32 fixed volume that requires grad."""
    if not ctx.needs_input_grad[1]:
        return None
    _, gf = ctx.plan.grad_fixed(fixed.detach(), moving, disp, dense=dense)
    return gf * grad_output.to(torch.float32)


class SRWCRLoss(torch.autograd.Function):
    """D = SRWCR as a differentiable function of the FFD displacements (and of
    the normalised fixed volume when it requires grad).

    forward runs srwcr_eval; backward runs srwcr_grad (and srwcr_grad_fixed)
    and scales by grad_output."""

    @staticmethod
    def forward(ctx, ffd, fixed, moving, plan):
        ctx.plan = plan
        ctx.save_for_backward(ffd, fixed, moving)
        return plan.eval(fixed.detach(), moving, ffd.detach().contiguous()).clone()

    @staticmethod
    def backward(ctx, grad_output):
        ffd, fixed, moving = ctx.saved_tensors
        d = ffd.detach().contiguous()
        g = None
        if ctx.needs_input_grad[0]:
            _, g = ctx.plan.grad(fixed.detach(), moving, d)
            g = g * grad_output.to(torch.float32)
        return g, _fixed_grad(ctx, d, fixed, moving, False, grad_output), None, None


class SRWCRDenseLoss(torch.autograd.Function):
    """D = SRWCR as a differentiable function of a dense displacement field
    u[3][nz][ny][nx] (T(x) = x + u(x)), e.g. the output of a registration
    network (and of the normalised fixed volume when it requires grad).
    backward runs srwcr_grad_dense (and srwcr_grad_fixed) and scales by
    grad_output."""

    @staticmethod
    def forward(ctx, field, fixed, moving, plan):
        ctx.plan = plan
        ctx.save_for_backward(field, fixed, moving)
        return plan.eval_dense(fixed.detach(), moving, field.detach().contiguous()).clone()

    @staticmethod
    def backward(ctx, grad_output):
        field, fixed, moving = ctx.saved_tensors
        u = field.detach().contiguous()
        g = None
        if ctx.needs_input_grad[0]:
            _, g = ctx.plan.grad_dense(fixed.detach(), moving, u)
            g = g * grad_output.to(torch.float32)
        return g, _fixed_grad(ctx, u, fixed, moving, True, grad_output), None, None
