"""Seeded synthetic volumes for the SRWCR workloads.

This module draws raw intensities only.  It holds none of the method's
arithmetic (no normalisation, no FFD evaluation, no Parzen window, no
histogram), so both the CPU oracle and the HIP path can consume its output.

Every generator uses ``numpy.random.default_rng(1804_05061 + k)`` for workload
k and draws in a fixed order, so a (workload, seed) pair always yields the same
arrays.  Volumes are float32 arrays shaped (nz, ny, nx), x fastest.
Deformations used to *make* a moving image are smooth random fields drawn on a
coarse grid and up-sampled by scipy's cubic-spline interpolation; they are an
input recipe and unrelated to the FFD the library evaluates.

Workloads (they stand in for the paper's synthetic grids, 4-D CT, OCT and
CT/PET data, which are not available):
  1  blobs 64^3, moving = blobs warped (spacing 8, N(0, 2 vox)) times a smooth
     bias field, N(0, 0.01) noise;                        32 bins, 4x4x4 regions
  2  CT-like 256x256x128 ellipsoid phantom (HU labels), moving warped by a
     breathing shift (max 15 vox, superior-inferior = z) plus a random field
     (spacing 10), N(0, 20 HU) noise;                     64 bins, 6x6x6 regions
  3  OCT-like 512x512x128 layered volume (8 smooth surfaces, depth = y),
     multiplicative Gamma(k=2, theta=0.5) speckle;        64 bins, 8x8x4 regions
  4  CT-like 192^3 fixed, PET-like 96^3 moving (non-monotone uptake map,
     Gaussian blur sigma 2, Poisson noise);               48 bins, 5x5x5 regions
  5  9 breathing phases of the workload-2 phantom, cropped to 80..128 slices.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy import ndimage

SEED_BASE = 1804_05061
HU_LABELS = np.array([-1000.0, -50.0, 40.0, 400.0, 1200.0])


@dataclass
class Workload:
    name: str
    fixed: np.ndarray            # float32 (nz, ny, nx)
    moving: np.ndarray           # float32 (mz, my, mx)
    n_bins: int
    spatial_bins: tuple          # (Kx, Ky, Kz)
    ctrl_spacing: tuple          # (dx, dy, dz)
    role: int = 0                # 0: moving is A (model image); 1: moving is B
    meta: dict = field(default_factory=dict)

    @property
    def fixed_dims(self):
        return tuple(int(v) for v in self.fixed.shape[::-1])

    @property
    def moving_dims(self):
        return tuple(int(v) for v in self.moving.shape[::-1])

    @property
    def ctrl_dims(self):
        return tuple((n - 1) // d + 4 for n, d in zip(self.fixed_dims, self.ctrl_spacing))


def rng_for(k: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + k + 1000 * salt)


def _spline_matrix(n_fine, n_coarse):
    """(n_fine, n_coarse) matrix of 1-D cubic-spline interpolation weights
    mapping a coarse grid spanning [0, n_fine - 1] onto the fine samples."""
    pos = np.linspace(0, n_coarse - 1, n_fine)
    W = np.empty((n_fine, n_coarse))
    for j in range(n_coarse):
        e = np.zeros(n_coarse)
        e[j] = 1.0
        W[:, j] = ndimage.map_coordinates(e, pos[None, :], order=3, mode="nearest")
    return W


def smooth_field(rng, shape, spacing, sigma, comps=3):
    """Random smooth vector field: N(0, sigma) values on a grid of the given
    spacing, up-sampled to `shape` (nz, ny, nx) by cubic-spline interpolation."""
    nz, ny, nx = shape
    cz, cy, cx = (max(2, int(np.ceil((n - 1) / spacing)) + 1) for n in (nz, ny, nx))
    Wz, Wy, Wx = _spline_matrix(nz, cz), _spline_matrix(ny, cy), _spline_matrix(nx, cx)
    out = np.empty((comps, nz, ny, nx), dtype=np.float32)
    for c in range(comps):
        coarse = rng.normal(0.0, sigma, size=(cz, cy, cx))
        a = np.einsum("zc,cyx->zyx", Wz, coarse)
        a = np.einsum("yc,zcx->zyx", Wy, a)
        out[c] = np.einsum("xc,zyc->zyx", Wx, a).astype(np.float32)
    return out


def _grid(shape):
    nz, ny, nx = shape
    z = np.arange(nz, dtype=np.float32)[:, None, None]
    y = np.arange(ny, dtype=np.float32)[None, :, None]
    x = np.arange(nx, dtype=np.float32)[None, None, :]
    return z, y, x


# ----------------------------------------------------------------- blobs
def blobs(n=64, k=1, n_blobs=12):
    """Workload 1: sum of Gaussian blobs, warped copy times a bias field."""
    rng = rng_for(k)
    shape = (n, n, n)
    centres = rng.uniform(0, n - 1, size=(n_blobs, 3))
    sigmas = rng.uniform(4, 10, size=n_blobs)
    amps = rng.uniform(0, 1, size=n_blobs)
    u = smooth_field(rng, shape, 8, 2.0)                       # x, y, z components
    bias = 1.0 + 0.2 * smooth_field(rng, shape, 32, 1.0, comps=1)[0].clip(-1, 1)
    z, y, x = _grid(shape)

    def render(xs, ys, zs):
        f = np.zeros(np.broadcast_shapes(xs.shape, ys.shape, zs.shape), dtype=np.float32)
        for (cx, cy, cz), s, a in zip(centres, sigmas, amps):
            d2 = (xs - cx) ** 2 + (ys - cy) ** 2 + (zs - cz) ** 2
            f += np.float32(a) * np.exp(-d2 / np.float32(2 * s * s))
        return f

    fixed = render(x, y, z) + rng.normal(0, 0.01, size=shape).astype(np.float32)
    moving = render(x + u[0], y + u[1], z + u[2]) * bias + rng.normal(0, 0.01, size=shape).astype(np.float32)
    return Workload("blobs64", fixed.astype(np.float32), moving.astype(np.float32), 32, (4, 4, 4), (8, 8, 8),
                    role=0, meta={"u": u})


# ------------------------------------------------------------ CT phantom
def _ellipsoids(rng, shape, n_ell=40):
    nz, ny, nx = shape
    ells = []
    lo = np.array([0.5 - 0.45, 0.5 - 0.35, 0.5 - 0.48]) * np.array([nx, ny, nz])
    hi = np.array([0.5 + 0.45, 0.5 + 0.35, 0.5 + 0.48]) * np.array([nx, ny, nz])
    for _ in range(n_ell):
        c = rng.uniform(lo, hi)
        ax = rng.uniform(4, 40, size=3)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        w, a, b, cc = q
        Rm = np.array([[1 - 2 * (b * b + cc * cc), 2 * (a * b - cc * w), 2 * (a * cc + b * w)],
                       [2 * (a * b + cc * w), 1 - 2 * (a * a + cc * cc), 2 * (b * cc - a * w)],
                       [2 * (a * cc - b * w), 2 * (b * cc + a * w), 1 - 2 * (a * a + b * b)]])
        lab = int(rng.integers(0, len(HU_LABELS)))
        ells.append((c, ax, Rm, lab))
    return ells


def _render_labels(ells, shape, xs, ys, zs):
    """Label volume (index into HU_LABELS, or -1 outside the body) at points."""
    nz, ny, nx = shape
    lab = np.full(np.broadcast_shapes(xs.shape, ys.shape, zs.shape), -1, dtype=np.int8)
    body = (((xs - 0.5 * nx) / (0.45 * nx)) ** 2 + ((ys - 0.5 * ny) / (0.35 * ny)) ** 2
            + ((zs - 0.5 * nz) / (0.48 * nz)) ** 2) <= 1.0
    lab[body] = 2                                                # 40 HU soft tissue
    zlo, zhi = float(np.min(zs)), float(np.max(zs))
    for c, ax, Rm, l in ells:
        rad = float(np.max(ax))
        if c[2] + rad < zlo or c[2] - rad > zhi:                 # slab misses the ellipsoid
            continue
        dx, dy, dz = xs - c[0], ys - c[1], zs - c[2]
        r0 = (Rm[0, 0] * dx + Rm[1, 0] * dy + Rm[2, 0] * dz) / ax[0]
        r1 = (Rm[0, 1] * dx + Rm[1, 1] * dy + Rm[2, 1] * dz) / ax[1]
        r2 = (Rm[0, 2] * dx + Rm[1, 2] * dy + Rm[2, 2] * dz) / ax[2]
        lab[(r0 * r0 + r1 * r1 + r2 * r2) <= 1.0] = l
    return lab


def _labels_to_hu(lab):
    hu = np.where(lab < 0, np.float32(-1000.0), HU_LABELS.astype(np.float32)[np.maximum(lab, 0)])
    return hu.astype(np.float32)


def breathing_field(shape, amplitude):
    """Smooth superior-inferior (z) shift, largest mid-volume at the centre."""
    nz, ny, nx = shape
    z, y, x = _grid(shape)
    xc, yc = 0.5 * (nx - 1), 0.5 * (ny - 1)
    uz = amplitude * np.sin(np.pi * z / max(nz - 1, 1)) * np.exp(
        -((x - xc) ** 2 + (y - yc) ** 2) / (2 * (0.3 * nx) ** 2))
    return uz.astype(np.float32)


def _render_slabwise(fn, shape, u, slab=16):
    """Evaluate fn(xs, ys, zs) at x + u(x) slab by slab (bounded memory)."""
    nz, ny, nx = shape
    out = None
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        z, y, x = _grid((z1 - z0, ny, nx))
        z = z + z0
        if u is not None:
            xs, ys, zs = x + u[0, z0:z1], y + u[1, z0:z1], z + u[2, z0:z1]
        else:
            xs, ys, zs = (np.broadcast_to(x, (z1 - z0, ny, nx)), np.broadcast_to(y, (z1 - z0, ny, nx)),
                          np.broadcast_to(z, (z1 - z0, ny, nx)))
        r = fn(xs, ys, zs)
        if out is None:
            out = np.empty((nz, ny, nx), dtype=r.dtype)
        out[z0:z1] = r
    return out


def ct_phantom(shape=(128, 256, 256), k=2, breathing=15.0, field_spacing=10, field_sigma=2.0,
               noise=20.0, with_moving=True):
    """Workload 2: CT-like label phantom (HU) and its breathing-warped copy."""
    rng = rng_for(k)
    ells = _ellipsoids(rng, shape)
    lab_f = _render_slabwise(lambda xs, ys, zs: _render_labels(ells, shape, xs, ys, zs), shape, None)
    fixed = _labels_to_hu(lab_f) + rng.normal(0, noise, size=shape).astype(np.float32)
    meta = {"labels": lab_f}
    moving = None
    if with_moving:
        u = smooth_field(rng, shape, field_spacing, field_sigma)
        u[2] += breathing_field(shape, breathing)
        lab_m = _render_slabwise(lambda xs, ys, zs: _render_labels(ells, shape, xs, ys, zs), shape, u)
        moving = _labels_to_hu(lab_m) + rng.normal(0, noise, size=shape).astype(np.float32)
        meta["u"] = u
        meta["ellipsoids"] = ells
    nz, ny, nx = shape
    return Workload(f"ct{nx}x{ny}x{nz}", fixed.astype(np.float32),
                    None if moving is None else moving.astype(np.float32), 64, (6, 6, 6), (10, 10, 10),
                    role=0, meta=meta)


# ------------------------------------------------------------------- OCT
def oct_layers(shape=(128, 512, 512), k=3):
    """Workload 3: layered OCT-like volume with gamma speckle (depth = y)."""
    rng = rng_for(k)
    nz, ny, nx = shape
    n_surf = 8
    base = np.sort(rng.uniform(0.25, 0.75, size=n_surf)) * ny
    for i in range(1, n_surf):                                   # minimum gap 3 vox
        base[i] = max(base[i], base[i - 1] + 3.0)
    zz = np.arange(nz, dtype=np.float32)[:, None]
    xx = np.arange(nx, dtype=np.float32)[None, :]
    surf = np.empty((n_surf, nz, nx), dtype=np.float32)
    for i in range(n_surf):
        s = np.full((nz, nx), base[i], dtype=np.float32)
        for _ in range(3):
            amp = rng.uniform(0, 10.0 / 3)
            fx, fz = rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0)
            ph = rng.uniform(0, 2 * np.pi)
            s += amp * np.sin(2 * np.pi * (fx * xx / nx + fz * zz / nz) + ph)
        surf[i] = s
    for i in range(1, n_surf):
        surf[i] = np.maximum(surf[i], surf[i - 1] + 3.0)
    inten = rng.uniform(0.05, 1.0, size=n_surf + 1).astype(np.float32)
    u = smooth_field(rng, shape, 16, 2.0)

    def render(xs, ys, zs):
        # layer index = number of surfaces above the point (nearest surface sample)
        xi = np.clip(np.rint(xs), 0, nx - 1).astype(np.int32)
        zi = np.clip(np.rint(zs), 0, nz - 1).astype(np.int32)
        layer = np.zeros(xs.shape, dtype=np.int32)
        for i in range(n_surf):
            layer += (ys >= surf[i][zi, xi]).astype(np.int32)
        return inten[layer]

    fixed = _render_slabwise(render, shape, None)
    moving = _render_slabwise(render, shape, u)
    fixed = fixed * rng.gamma(2.0, 0.5, size=shape).astype(np.float32)
    moving = moving * rng.gamma(2.0, 0.5, size=shape).astype(np.float32)
    return Workload(f"oct{nx}x{ny}x{nz}", fixed.astype(np.float32), moving.astype(np.float32), 64, (8, 8, 4),
                    (16, 16, 16), role=0, meta={"u": u})


# ---------------------------------------------------------------- CT/PET
def ct_pet(n=192, k=4):
    """Workload 4: CT-like fixed n^3, PET-like moving (n/2)^3 with a non-monotone uptake map."""
    rng = rng_for(k)
    shape = (n, n, n)
    ells = _ellipsoids(rng, shape)
    lab_f = _render_slabwise(lambda xs, ys, zs: _render_labels(ells, shape, xs, ys, zs), shape, None)
    fixed = _labels_to_hu(lab_f) + rng.normal(0, 20.0, size=shape).astype(np.float32)
    while True:                                                   # reject monotone maps
        uptake = rng.uniform(0, 1, size=len(HU_LABELS) + 1)
        d = np.diff(uptake[1:])
        if not (np.all(d > 0) or np.all(d < 0)):
            break
    u = smooth_field(rng, shape, 8, 2.0)
    lab_m = _render_slabwise(lambda xs, ys, zs: _render_labels(ells, shape, xs, ys, zs), shape, u)
    up = uptake[lab_m.astype(np.int32) + 1].astype(np.float32)    # index 0 = outside the body
    m = n // 2
    up = up.reshape(m, 2, m, 2, m, 2).mean(axis=(1, 3, 5))
    up = ndimage.gaussian_filter(up, 2.0)
    moving = rng.poisson(50.0 * np.maximum(up, 0)).astype(np.float32) / 50.0
    return Workload(f"ctpet{n}to{m}", fixed.astype(np.float32), moving.astype(np.float32), 48, (5, 5, 5),
                    (8, 8, 8), role=0, meta={"u": u, "uptake": uptake})


# ----------------------------------------------------------- 4-D phases
def _phase_labels(ells, shape, amp):
    """Label volume of one breathing phase (amp None: the reference phase)."""
    u = None
    if amp is not None:
        u = np.zeros((3,) + tuple(shape), dtype=np.float32)
        u[2] = breathing_field(shape, amp)
    return _render_slabwise(lambda xs, ys, zs: _render_labels(ells, shape, xs, ys, zs), shape, u)


def breathing_phases(shape=(128, 256, 256), k=5, n_phases=9, workers=1, mp_context="fork"):
    """Workload 5: phase 0 and phases 1..9 of a breathing cycle, pair k cropped
    to the centre (80 + 6 (k - 1)) / 128 of the slices.  Returns a list of
    (fixed, moving) raw pairs.  `workers` > 1 renders the phases in worker
    processes of `mp_context` (the random draws stay in the calling process,
    in order); "spawn" suits a caller that already holds a GPU."""
    rng = rng_for(k)
    ells = _ellipsoids(rng, shape)
    nz = shape[0]
    amps = [None] + [3.0 + 12.0 * (ph - 1) / (n_phases - 1) for ph in range(1, n_phases + 1)]
    if workers > 1:
        import multiprocessing
        with multiprocessing.get_context(mp_context).Pool(min(workers, len(amps))) as pool:
            labs = pool.starmap(_phase_labels, [(ells, shape, a) for a in amps])
    else:
        labs = [_phase_labels(ells, shape, a) for a in amps]
    fixed_full = _labels_to_hu(labs[0]) + rng.normal(0, 20.0, size=shape).astype(np.float32)
    pairs = []
    for ph in range(1, n_phases + 1):
        mov = _labels_to_hu(labs[ph]) + rng.normal(0, 20.0, size=shape).astype(np.float32)
        zk = nz * (80 + 6 * (ph - 1)) // 128      # 80, 86, ..., 128 slices of 128
        z0 = (nz - zk) // 2
        pairs.append((np.ascontiguousarray(fixed_full[z0:z0 + zk]), np.ascontiguousarray(mov[z0:z0 + zk])))
    return pairs


def pyramid(vol, levels=3):
    """Input pyramid of workload 5: level 0 is `vol`, each next level a
    Gaussian (sigma 1 voxel) of the previous one at every second voxel."""
    out = [np.ascontiguousarray(vol)]
    for _ in range(levels - 1):
        out.append(np.ascontiguousarray(ndimage.gaussian_filter(out[-1], 1.0)[::2, ::2, ::2]))
    return out


def breathing4d_ffd(ctrl_dims, pair, level):
    """Displacements of problem (pair, level) of workload 5: N(0, 2 vox)."""
    return random_ffd(ctrl_dims, 2.0, 5, salt=10 * pair + level)


def random_ffd(ctrl_dims, sigma, k, salt=7):
    """Seeded FFD displacements (3, ncz, ncy, ncx), N(0, sigma) voxels."""
    rng = rng_for(k, salt)
    ncx, ncy, ncz = ctrl_dims
    return rng.normal(0.0, sigma, size=(3, ncz, ncy, ncx)).astype(np.float32)


def smooth_pair(shape, k=0, n_blobs=6):
    """Small smooth blob volumes for finite-difference checks (16^3 and such)."""
    rng = rng_for(k, 3)
    nz, ny, nx = shape
    z, y, x = _grid(shape)
    f = np.zeros(shape, dtype=np.float64)
    g = np.zeros(shape, dtype=np.float64)
    for _ in range(n_blobs):
        c = rng.uniform(0, 1, size=3) * np.array([nx - 1, ny - 1, nz - 1])
        s = rng.uniform(2.0, 5.0)
        a, b = rng.uniform(0.2, 1.0, size=2)
        e = np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * s * s))
        f += a * e
        g += b * np.exp(-((x - c[0] - 0.7) ** 2 + (y - c[1] + 0.4) ** 2 + (z - c[2]) ** 2) / (2 * s * s))
    return f.astype(np.float32), g.astype(np.float32)


def raptor_patches(fixed_dims, side=17, coverage=1.0, k=0, extra_edge=True):
    """Seeded RaPTOR patches: int32 [n, 6] half-open cubes (x0, y0, z0, x1,
    y1, z1) of `side` voxels, centres uniform over the fixed grid (the boxes
    reach past the border there and are clipped by the method), n chosen so
    the patches hold `coverage` times the grid's voxel count.  With
    extra_edge, two more boxes are appended: one wholly outside the grid and
    one that covers it entirely."""
    rng = rng_for(k, 11)
    nx, ny, nz = fixed_dims
    n = max(1, int(round(coverage * nx * ny * nz / side ** 3)))
    c = np.stack([rng.integers(0, d, size=n) for d in (nx, ny, nz)], axis=1)
    lo = c - side // 2
    boxes = np.concatenate([lo, lo + side], axis=1)
    if extra_edge:
        boxes = np.concatenate([boxes, [[nx + 3, 0, 0, nx + 9, ny, nz], [-2, -2, -2, nx + 2, ny + 2, nz + 2]]])
    return boxes.astype(np.int32)
