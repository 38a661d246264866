"""Python access to the FP64 CPU oracle (``srwcr_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.  It shares no code
with the HIP path.  Each function states the passage of Gong et al. (arXiv
1804.05061) it follows; the arithmetic itself lives in the C file.

Volumes are numpy arrays shaped (nz, ny, nx) (x fastest in memory); FFD
displacements are float32 arrays shaped (3, ncz, ncy, ncx), component 0 = x.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "srwcr_oracle.c")
# ORC_LIB names another build of the oracle (the sanitizer build of the
# tests); by default the one next to this file.
_LIB_PATH = os.environ.get("ORC_LIB") or os.path.join(_HERE, "liborc.so")


def build(force: bool = True, out: str = None, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FP contraction);
    sanitize: with AddressSanitizer and UndefinedBehaviorSanitizer, into `out`."""
    out = out or _LIB_PATH
    if force or not os.path.exists(out):
        san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"] \
            if sanitize else []
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", *san,
               "-o", out + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return out


class _Problem(ctypes.Structure):
    _fields_ = [("nf", ctypes.c_int * 3), ("nm", ctypes.c_int * 3), ("n_bins", ctypes.c_int),
                ("K", ctypes.c_int * 3), ("delta", ctypes.c_int * 3), ("role", ctypes.c_int),
                ("dense", ctypes.c_int), ("at_nodes", ctypes.c_int)]


@dataclass(frozen=True)
class Problem:
    """Problem statement of Sec. II: grids, L_eps + 1 bins, spatial bins, control spacing.

    role 0: the moving image plays A (the model image); role 1: it plays B
    (the estimated image) -- Sec. II-E / Table II.  spatial_bins == (1, 1, 1)
    selects one constant region (a test-only special case); (0, 0, 0) puts
    the regions on the FFD nodes, K = n_c per axis (the paper's setting, Sec. II-C).  dense: the
    displacements are a dense field u (3, nz, ny, nx) on the fixed grid,
    T(x) = x + u(x), instead of FFD coefficients."""
    fixed_dims: tuple   # (nx, ny, nz)
    moving_dims: tuple
    n_bins: int
    spatial_bins: tuple
    ctrl_spacing: tuple
    role: int
    dense: bool = False

    def c(self) -> _Problem:
        p = _Problem()
        p.nf[:] = list(self.fixed_dims)
        p.nm[:] = list(self.moving_dims)
        p.n_bins = self.n_bins
        p.K[:] = list(self.ctrl_dims if self.at_nodes else self.spatial_bins)
        p.at_nodes = 1 if self.at_nodes else 0
        p.delta[:] = list(self.ctrl_spacing)
        p.role = self.role
        p.dense = 1 if self.dense else 0
        return p

    @property
    def ctrl_dims(self) -> tuple:
        """n_c = floor((N - 1) / delta) + 4 per axis (eq 17 indexing), (ncx, ncy, ncz)."""
        return tuple((n - 1) // d + 4 for n, d in zip(self.fixed_dims, self.ctrl_spacing))

    @property
    def n_regions(self) -> int:
        return int(np.prod(self.ctrl_dims if self.at_nodes else self.spatial_bins))

    @property
    def at_nodes(self) -> bool:
        """spatial_bins == (0, 0, 0): the regions are the FFD nodes (the paper's setting)."""
        return tuple(self.spatial_bins) == (0, 0, 0)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        pp = ctypes.POINTER(_Problem)
        L.orc_h.restype = ctypes.c_double
        L.orc_h.argtypes = [ctypes.c_double]
        L.orc_dh.restype = ctypes.c_double
        L.orc_dh.argtypes = [ctypes.c_double, ctypes.c_int]
        L.orc_beta.restype = ctypes.c_double
        L.orc_beta.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_normalize.restype = None
        L.orc_normalize.argtypes = [fp, ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_int, fp]
        L.orc_axis_region_weights.restype = None
        L.orc_axis_region_weights.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.orc_axis_node_weights.restype = None
        L.orc_axis_node_weights.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.orc_ffd_T.restype = None
        L.orc_ffd_T.argtypes = [pp, fp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.orc_sample.restype = ctypes.c_double
        L.orc_sample.argtypes = [pp, fp, dp, dp]
        L.orc_warp.restype = None
        L.orc_warp.argtypes = [pp, fp, fp, dp]
        L.orc_joint_pdf.restype = ctypes.c_double
        L.orc_joint_pdf.argtypes = [pp, fp, fp, fp, dp]
        L.orc_joint_mass_box.restype = None
        L.orc_joint_mass_box.argtypes = [pp, fp, fp, fp, ctypes.POINTER(ctypes.c_int), dp]
        L.orc_srwcr_from_pdf.restype = ctypes.c_double
        L.orc_srwcr_from_pdf.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int]
        L.orc_value.restype = ctypes.c_double
        L.orc_value.argtypes = [pp, fp, fp, fp]
        L.orc_gradient.restype = ctypes.c_double
        L.orc_gradient.argtypes = [pp, fp, fp, fp, ctypes.c_int, dp, dp]
        L.orc_gradient_fixed.restype = ctypes.c_double
        L.orc_gradient_fixed.argtypes = [pp, fp, fp, fp, ctypes.c_int, dp]
        L.orc_raptor.restype = ctypes.c_double
        L.orc_raptor.argtypes = [pp, fp, fp, fp, ctypes.POINTER(ctypes.c_int), ctypes.c_int, dp, dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _f64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def h(t: float) -> float:
    """Second-order Parzen window, eq (5)."""
    return lib().orc_h(float(t))


def dh(kappa: float, side: int) -> float:
    """dh/dkappa; side -1 left derivative, +1 right derivative."""
    return lib().orc_dh(float(kappa), int(side))


def beta(l: int, t: float) -> float:
    """Cubic B-spline piece beta_l(t), eq (8)."""
    return lib().orc_beta(int(l), float(t))


def normalize(raw: np.ndarray, lo: float, hi: float, n_bins: int) -> np.ndarray:
    """Linear min-max normalisation to [0, L_eps] (Sec. II), FP32 arithmetic."""
    a, ptr = _f32(raw)
    out = np.empty_like(a)
    lib().orc_normalize(ptr, a.size, float(lo), float(hi), int(n_bins), _f32(out)[1])
    return out


def axis_region_weights(x: int, N: int, K: int) -> np.ndarray:
    """Spatial weights of the K nodes of one axis at voxel x, eqs (7, 8)."""
    w = np.zeros(K, dtype=np.float64)
    lib().orc_axis_region_weights(int(x), int(N), int(K), _f64(w))
    return w


def axis_node_weights(x: int, delta: int, K: int) -> np.ndarray:
    """Spatial weights of the K FFD-lattice nodes of one axis at voxel x (regions
    at the control points, Sec. II-C)."""
    w = np.zeros(K, dtype=np.float64)
    lib().orc_axis_node_weights(int(x), int(delta), int(K), _f64(w))
    return w


def ffd_T(P: Problem, ffd: np.ndarray, x: int, y: int, z: int) -> np.ndarray:
    """T(x; Phi) at one fixed voxel, eqs (8, 17)."""
    f, fp = _f32(ffd)
    T = np.zeros(3)
    lib().orc_ffd_T(ctypes.byref(P.c()), fp, x, y, z, _f64(T))
    return T


def sample(P: Problem, moving: np.ndarray, y) -> tuple:
    """Trilinear sample of the moving volume at moving-grid coordinates y; returns (value, dM/dy)."""
    m, mp = _f32(moving)
    yy = np.asarray(y, dtype=np.float64).copy()
    g = np.zeros(3)
    v = lib().orc_sample(ctypes.byref(P.c()), mp, _f64(yy), _f64(g))
    return v, g


def warp(P: Problem, moving: np.ndarray, ffd: np.ndarray) -> np.ndarray:
    """Backward-warped moving intensity at every fixed voxel (Sec. II-F)."""
    m, mp = _f32(moving)
    f, fp = _f32(ffd)
    nx, ny, nz = P.fixed_dims
    out = np.zeros((nz, ny, nx))
    lib().orc_warp(ctypes.byref(P.c()), mp, fp, _f64(out))
    return out


def joint_pdf(P: Problem, fixed: np.ndarray, moving: np.ndarray, ffd: np.ndarray):
    """Normalised 3-D joint PDF p[r, a, b] of eq (3) and its normaliser Z."""
    fx, fxp = _f32(fixed)
    m, mp = _f32(moving)
    f, fp = _f32(ffd)
    p = np.zeros((P.n_regions, P.n_bins, P.n_bins))
    Z = lib().orc_joint_pdf(ctypes.byref(P.c()), fxp, mp, fp, _f64(p))
    return p, Z


def joint_mass_box(P: Problem, fixed: np.ndarray, moving: np.ndarray, ffd: np.ndarray, box,
                   q: np.ndarray | None = None) -> np.ndarray:
    """Unnormalised eq (3) mass of the voxels in box = (x0, x1, y0, y1, z0, z1)
    (half-open), added to q[r, a, b] (a new zero array when q is None)."""
    fx, fxp = _f32(fixed)
    m, mp = _f32(moving)
    f, fp = _f32(ffd)
    if q is None:
        q = np.zeros((P.n_regions, P.n_bins, P.n_bins))
    assert q.dtype == np.float64 and q.flags.c_contiguous and q.shape == (P.n_regions, P.n_bins, P.n_bins)
    b = (ctypes.c_int * 6)(*[int(v) for v in box])
    lib().orc_joint_mass_box(ctypes.byref(P.c()), fxp, mp, fp, b, _f64(q))
    return q


def node_support_box(P: Problem, node) -> tuple:
    """Fixed voxels whose warp T (eq 17, stored node index = paper index + 1)
    involves control node (i, j, k): floor(x / delta) in [i - 3, i] per axis.
    For a dense field, (i, j, k) is a voxel and its box is that voxel."""
    if P.dense:
        i, j, k = node
        return (i, i + 1, j, j + 1, k, k + 1)
    box = []
    for n, d, N in zip(node, P.ctrl_spacing, P.fixed_dims):
        box += [max(0, (n - 3) * d), min(N, (n + 1) * d)]
    return tuple(box)


def fd_control_points(P: Problem, fixed: np.ndarray, moving: np.ndarray, ffd: np.ndarray, points,
                      h: float, threads: int | None = None) -> np.ndarray:
    """Central finite differences of D (eq 9, Table I loop) with respect to
    single displacement components points = [(e, k, j, i), ...] (component e
    of stored node (i, j, k), or of voxel (i, j, k) of a dense field).

    Eq (3) is a sum over voxels, so the perturbed Z p is the unperturbed Z p
    minus the old and plus the new mass of the voxels whose warp the node
    changes; D+ and D- are then computed from their normalised PDFs.  The step
    is the one float32 storage actually takes: (d + h) - (d - h) after rounding."""
    from concurrent.futures import ThreadPoolExecutor
    ffd = np.ascontiguousarray(ffd, dtype=np.float32)
    p, Z = joint_pdf(P, fixed, moving, ffd)
    q_full = p * Z

    def one(pt):
        e, k, j, i = pt
        box = node_support_box(P, (i, j, k))
        q_rest = q_full - joint_mass_box(P, fixed, moving, ffd, box)
        Ds, steps = [], []
        for sgn in (+1.0, -1.0):
            f2 = ffd.copy()
            f2[e, k, j, i] = np.float32(float(ffd[e, k, j, i]) + sgn * h)
            steps.append(float(f2[e, k, j, i]))
            q = joint_mass_box(P, fixed, moving, f2, box, q_rest.copy())
            Ds.append(srwcr_from_pdf(q / q.sum()))
        return (Ds[0] - Ds[1]) / (steps[0] - steps[1])

    with ThreadPoolExecutor(max_workers=threads or os.cpu_count() or 1) as ex:
        return np.array(list(ex.map(one, list(points))))


def srwcr_from_pdf(p: np.ndarray, which: int = 0) -> float:
    """SRWCR from a joint PDF: 0 Table I loop, 1 eq (9), 2 eq (11), 3 eq (12)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    R, nb, _ = p.shape
    return lib().orc_srwcr_from_pdf(R, nb, _f64(p), int(which))


def value(P: Problem, fixed: np.ndarray, moving: np.ndarray, ffd: np.ndarray) -> float:
    """D = SRWCR(A, B, R), eq (9) evaluated by the Table I loop."""
    fx, fxp = _f32(fixed)
    m, mp = _f32(moving)
    f, fp = _f32(ffd)
    return lib().orc_value(ctypes.byref(P.c()), fxp, mp, fp)


def gradient(P: Problem, fixed: np.ndarray, moving: np.ndarray, ffd: np.ndarray,
             form: int = 0, want_dDdM: bool = False):
    """(D, dD/d(displacement)[3, ncz, ncy, ncx]) by eqs (16, 17) with dD/dM from
    eq (19)/(21) (form 0) or eq (18)/(20) + (26) (form 1).  For a dense field
    (P.dense) the gradient is dD/du[3, nz, ny, nx], eq (16) per voxel."""
    fx, fxp = _f32(fixed)
    m, mp = _f32(moving)
    f, fp = _f32(ffd)
    ncx, ncy, ncz = P.ctrl_dims
    nx, ny, nz = P.fixed_dims
    g = np.zeros((3, nz, ny, nx)) if P.dense else np.zeros((3, ncz, ncy, ncx))
    dm = np.zeros((nz, ny, nx)) if want_dDdM else None
    D = lib().orc_gradient(ctypes.byref(P.c()), fxp, mp, fp, int(form), _f64(g),
                           _f64(dm) if dm is not None else None)
    return (D, g, dm) if want_dDdM else (D, g)


def gradient_fixed(P: Problem, fixed: np.ndarray, moving: np.ndarray, disp: np.ndarray, form: int = 0):
    """(D, dD/ds_F[nz, ny, nx]): the derivative of D with respect to the
    normalised fixed intensity at every voxel (eq 19 or 21 for the fixed
    image's role; form 1: eqs 18/20 with 26)."""
    fx, fxp = _f32(fixed)
    m, mp = _f32(moving)
    f, fp = _f32(disp)
    nx, ny, nz = P.fixed_dims
    g = np.zeros((nz, ny, nx))
    D = lib().orc_gradient_fixed(ctypes.byref(P.c()), fxp, mp, fp, int(form), _f64(g))
    return D, g


def raptor(P: Problem, fixed: np.ndarray, moving: np.ndarray, disp: np.ndarray, patches,
           want_grad: bool = False, want_dRds: bool = False):
    """RaPTOR of eqs (13, 14) over boxcar patches (eq 6), patches = int array
    [n, 6] of half-open boxes (x0, y0, z0, x1, y1, z1); linear window on A,
    frequency moments of B.  Returns the value, plus dRaPTOR/d(displacement)
    (FFD or dense layout as in gradient()) and dRaPTOR/ds_M per voxel when asked."""
    fx, fxp = _f32(fixed)
    m, mp = _f32(moving)
    f, fp = _f32(disp)
    pt = np.ascontiguousarray(patches, dtype=np.int32).reshape(-1, 6)
    ptp = pt.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    nx, ny, nz = P.fixed_dims
    ncx, ncy, ncz = P.ctrl_dims
    g = None
    if want_grad:
        g = np.zeros((3, nz, ny, nx)) if P.dense else np.zeros((3, ncz, ncy, ncx))
    d = np.zeros((nz, ny, nx)) if want_dRds else None
    v = lib().orc_raptor(ctypes.byref(P.c()), fxp, mp, fp, ptp, len(pt), _f64(g) if g is not None else None,
                         _f64(d) if d is not None else None)
    out = [v]
    if want_grad:
        out.append(g)
    if want_dRds:
        out.append(d)
    return out[0] if len(out) == 1 else tuple(out)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (for timing)."""
    lib().orc_set_num_threads(int(n))
