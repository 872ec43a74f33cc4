"""Seeded synthetic inputs for the solar-tomography workloads.

This module only *describes* inputs: the voxel grid, the observers and their
detector frames, Gaussian-blob phantoms, masks and noise.  It holds none of
the projector's or the solver's arithmetic, so both the FP64 oracle and the
GPU library can consume its output without sharing any method code.

Geometry conventions (the paper, Sec. "Instrument Independence", says only
that WCS keywords define the observer and the projector; these are the
readings used throughout):

* Cube frame: x toward heliographic longitude 0 / latitude 0, y toward
  longitude 90 deg, z toward solar north.  Lengths in solar radii (R_sun).
* A view is a pinhole observer ``obs`` with an orthonormal detector frame:
  ``w`` points at the box centre, ``u = unit(w x z)`` is image +column (solar
  west), ``v = u x w`` is image +row (north).  The ray through pixel
  (col, row) has direction ``w + (col - crpix0) cdelt0 u + (row - crpix1)
  cdelt1 v`` (gnomonic / TAN), with 0-based pixel centres.
* A field of view F (in R_sun, measured at the observer distance D) over
  n pixels gives ``cdelt = F / (n D)`` radians per pixel and
  ``crpix = (n - 1) / 2``.

A view is stored as 16 float64 numbers: obs[3], w[3], u[3], v[3], cdelt[2],
crpix[2]; its pixel counts as (ncol, nrow).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

R_OBS = 215.0  # observer distance, R_sun (about 1 AU)
ROT_DEG_PER_DAY = 13.2  # solar rotation seen by the observer


@dataclass
class Geometry:
    """Voxel grid plus the stacked detector views that see it."""

    n: tuple  # (nx, ny, nz)
    lo: np.ndarray  # (3,) box lower corner
    hi: np.ndarray  # (3,) box upper corner
    views: np.ndarray  # (V, 16) float64
    npix: np.ndarray  # (V, 2) int32 (ncol, nrow)
    view_frame: Optional[np.ndarray] = None  # (V,) int32 frame of each view
    nframes: int = 1
    data_mask: Optional[np.ndarray] = None  # (sum ncol*nrow,) uint8, 1 = keep
    map_mask: Optional[np.ndarray] = None  # (nz, ny, nx) uint8, 1 = keep
    obstacle: Optional[np.ndarray] = None  # (cx, cy, cz, R): opaque sphere ending every line of sight
    gains: Optional[np.ndarray] = None  # (V,) float64 gain of the instrument that took each view

    @property
    def nviews(self) -> int:
        return int(self.views.shape[0])

    @property
    def nvox(self) -> int:
        nx, ny, nz = self.n
        return int(nx) * int(ny) * int(nz)

    @property
    def nrays(self) -> int:
        return int(np.sum(self.npix[:, 0].astype(np.int64) * self.npix[:, 1]))

    def view_offsets(self) -> np.ndarray:
        sizes = self.npix[:, 0].astype(np.int64) * self.npix[:, 1]
        return np.concatenate([[0], np.cumsum(sizes)])

    def cube_shape(self) -> tuple:
        nx, ny, nz = self.n
        if self.nframes > 1:
            return (self.nframes, nz, ny, nx)
        return (nz, ny, nx)

    def subset(self, view_ids) -> "Geometry":
        """Geometry restricted to some views (masks sliced to match)."""
        view_ids = np.asarray(view_ids, dtype=np.int64)
        dm = None
        if self.data_mask is not None:
            off = self.view_offsets()
            dm = np.concatenate([self.data_mask[off[v]:off[v + 1]] for v in view_ids])
        vf = None if self.view_frame is None else self.view_frame[view_ids].copy()
        return Geometry(self.n, self.lo.copy(), self.hi.copy(), self.views[view_ids].copy(),
                        self.npix[view_ids].copy(), vf, self.nframes, dm,
                        None if self.map_mask is None else self.map_mask.copy(),
                        None if self.obstacle is None else np.array(self.obstacle, dtype=np.float64),
                        None if self.gains is None else np.asarray(self.gains, dtype=np.float64)[view_ids].copy())


# ------------------------------------------------------------------ views


def observer(lon_deg: float, lat_deg: float = 0.0, dist: float = R_OBS) -> np.ndarray:
    lon, lat = np.deg2rad(lon_deg), np.deg2rad(lat_deg)
    return dist * np.array([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)])


def pinhole_view(obs, target=(0.0, 0.0, 0.0), npix=(32, 32), fov=3.2) -> tuple:
    """Detector frame of an observer looking at ``target`` with the given
    pixel counts and field of view (R_sun at the target distance)."""
    obs = np.asarray(obs, dtype=np.float64)
    w = np.asarray(target, dtype=np.float64) - obs
    dist = np.linalg.norm(w)
    w = w / dist
    u = np.cross(w, [0.0, 0.0, 1.0])
    u = u / np.linalg.norm(u)
    v = np.cross(u, w)
    ncol, nrow = int(npix[0]), int(npix[1])
    cd = fov / (max(ncol, nrow) * dist)
    row = np.concatenate([obs, w, u, v, [cd, cd], [(ncol - 1) / 2.0, (nrow - 1) / 2.0]])
    return row, np.array([ncol, nrow], dtype=np.int32)


def make_views(lons, npix, fov, lat=0.0, dist=R_OBS):
    rows, pix = [], []
    for lon in lons:
        r, p = pinhole_view(observer(lon, lat, dist), npix=npix, fov=fov)
        rows.append(r)
        pix.append(p)
    return np.array(rows, dtype=np.float64), np.array(pix, dtype=np.int32)


def box(n: int, half: float) -> tuple:
    return (n, n, n), np.full(3, -half), np.full(3, half)


# --------------------------------------------------------------- phantoms


def voxel_centres(n, lo, hi):
    """Coordinates (z, y, x order of the arrays) of every voxel centre."""
    nx, ny, nz = n
    ax = [lo[a] + (np.arange(m) + 0.5) * (hi[a] - lo[a]) / m for a, m in enumerate((nx, ny, nz))]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return x, y, z


def draw_blobs(rng, nblobs, centre_range=1.2, sigma=(0.05, 0.3), amp=(0.0, 1.0)):
    """Blob parameters drawn per blob in the order (mu_x, mu_y, mu_z, sigma, a)."""
    out = np.empty((nblobs, 5))
    for b in range(nblobs):
        out[b, 0:3] = rng.uniform(-centre_range, centre_range, 3)
        out[b, 3] = rng.uniform(*sigma)
        out[b, 4] = rng.uniform(*amp)
    return out


def draw_shell_blobs(rng, nblobs, r_range=(1.5, 3.5), sigma=(0.1, 0.6), amp=(0.0, 1.0)):
    """Blobs at radius r ~ U(r_range) in isotropic random directions."""
    out = np.empty((nblobs, 5))
    for b in range(nblobs):
        r = rng.uniform(*r_range)
        dvec = rng.normal(size=3)
        dvec /= np.linalg.norm(dvec)
        out[b, 0:3] = r * dvec
        out[b, 3] = rng.uniform(*sigma)
        out[b, 4] = rng.uniform(*amp)
    return out


def blob_cube(n, lo, hi, blobs, rot_z_deg: float = 0.0) -> np.ndarray:
    """Sum of Gaussian blobs a exp(-|c - mu|^2 / 2 sigma^2) at voxel centres,
    optionally with the blob centres rotated about z."""
    nx, ny, nz = n
    ax = [lo[a] + (np.arange(m) + 0.5) * (hi[a] - lo[a]) / m for a, m in enumerate((nx, ny, nz))]
    out = np.zeros((nz, ny, nx))
    c, s = np.cos(np.deg2rad(rot_z_deg)), np.sin(np.deg2rad(rot_z_deg))
    for mx, my, mz, sg, a in blobs:
        rx, ry = c * mx - s * my, s * mx + c * my
        # exp of a sum of squares = product of per-axis factors
        k = 1.0 / (2.0 * sg * sg)
        gx, gy, gz = (np.exp(-((ax[i] - m) ** 2) * k) for i, m in enumerate((rx, ry, mz)))
        out += a * gz[:, None, None] * (gy[:, None] * gx[None, :])[None]
    return out


def radial_cube(n, lo, hi, power=8.0) -> np.ndarray:
    """r^-power outside the unit sphere, 0 inside."""
    x, y, z = voxel_centres(n, lo, hi)
    r = np.sqrt(x * x + y * y + z * z)
    out = np.zeros(r.shape)
    out[r >= 1.0] = r[r >= 1.0] ** (-power)
    return out


def sphere_map_mask(n, lo, hi, radius=1.0) -> np.ndarray:
    """1 where the voxel centre lies at r >= radius (kept), 0 inside."""
    x, y, z = voxel_centres(n, lo, hi)
    return (np.sqrt(x * x + y * y + z * z) >= radius).astype(np.uint8)


def annulus_data_mask(views, npix, rmin, rmax) -> np.ndarray:
    """1 for pixels whose impact radius on the plane of the sky (tangent-plane
    angle times observer distance) lies in [rmin, rmax]."""
    out = []
    for row16, (ncol, nrow) in zip(views, npix):
        dist = np.linalg.norm(row16[0:3])
        cols = (np.arange(ncol) - row16[14]) * row16[12]
        rows = (np.arange(nrow) - row16[15]) * row16[13]
        rr = np.hypot(cols[None, :], rows[:, None]) * dist
        out.append(((rr >= rmin) & (rr <= rmax)).astype(np.uint8).ravel())
    return np.concatenate(out)


def gaussian_noise(shape, sigma, seed) -> np.ndarray:
    return np.random.default_rng(seed).normal(0.0, sigma, shape)


def random_pair(nvox, nrays, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(size=nvox), rng.normal(size=nrays)


# ---------------------------------------------------------------- configs


@dataclass
class Workload:
    name: str
    geom: Geometry
    x: np.ndarray  # phantom, float64, shape geom.cube_shape()
    lam_r: float = 1e-2
    lam_t: float = 0.0
    cg_iters: int = 0
    noise_rel: float = 0.0
    noise_seed: Optional[int] = None
    extra: dict = field(default_factory=dict)


def tiny(seed: int = 0) -> Workload:
    """32^3 cube on [-1.5, 1.5]^3 with 16 blobs; 8 views 45 deg apart,
    32x32 pixels, FOV 3.2; 20 CG iterations at lambda 1e-2."""
    n, lo, hi = box(32, 1.5)
    views, npix = make_views([45.0 * k for k in range(8)], (32, 32), 3.2)
    blobs = draw_blobs(np.random.default_rng(seed), 16)
    g = Geometry(n, lo, hi, views, npix)
    return Workload("tiny-32^3-8x32^2", g, blob_cube(n, lo, hi, blobs), 1e-2, 0.0, 20)


def euvi_views(npix=512, fov=3.4, days=14):
    lons = []
    for k in range(days):
        lons.append(45.0 - ROT_DEG_PER_DAY * k)  # observer A
        lons.append(-45.0 - ROT_DEG_PER_DAY * k)  # observer B
    return make_views(lons, (npix, npix), fov)


def euvi(n: int = 128, npix: int = 512, seed: int = 1, noise_seed: int = 2) -> Workload:
    """EUVI-like static inversion: n^3 cube on [-1.5, 1.5]^3 with the unit
    sphere masked out; 28 views from two observers at +-45 deg rotated over
    14 days; blob + r^-8 phantom; 1% noise; 50 CG iterations at 1e-2."""
    nn, lo, hi = box(n, 1.5)
    views, pix = euvi_views(npix, 3.4)
    mm = sphere_map_mask(nn, lo, hi)
    blobs = draw_blobs(np.random.default_rng(seed), 16)
    x = (blob_cube(nn, lo, hi, blobs) + radial_cube(nn, lo, hi)) * mm
    g = Geometry(nn, lo, hi, views, pix, map_mask=mm)
    return Workload(f"euvi-{n}^3-28x{npix}^2", g, x, 1e-2, 0.0, 50, 0.01, noise_seed)


def differentiable(n: int = 128, npix: int = 256, nviews: int = 32) -> Workload:
    """128^3 cube, 32 views equally spaced in longitude, 256^2 pixels."""
    nn, lo, hi = box(n, 1.5)
    views, pix = make_views([360.0 * k / nviews for k in range(nviews)], (npix, npix), 3.4)
    x = blob_cube(nn, lo, hi, draw_blobs(np.random.default_rng(400), 16))
    target = blob_cube(nn, lo, hi, draw_blobs(np.random.default_rng(402), 16))
    g = Geometry(nn, lo, hi, views, pix)
    return Workload(f"autograd-{n}^3-{nviews}x{npix}^2", g, x, 1e-2, extra={"target_cube": target})


def learned(seed: int, n: int = 128, npix: int = 256) -> Workload:
    """Learned-preconditioner problem: n^3 blob phantom, the 28 EUVI-like
    views at npix^2, 1% noise, lambda 1e-2."""
    nn, lo, hi = box(n, 1.5)
    views, pix = euvi_views(npix, 3.4)
    x = blob_cube(nn, lo, hi, draw_blobs(np.random.default_rng(seed), 16))
    g = Geometry(nn, lo, hi, views, pix)
    return Workload(f"learned-{n}^3-seed{seed}", g, x, 1e-2, 0.0, 0, 0.01, seed + 7919)


def cor1_frames(n: int = 256, K: int = 8, npix: int = 512, nsteps: int = 30) -> Workload:
    """COR1-like time-evolving model: K frames of n^3 on [-4, 4]^3; 60 views
    (two observers at +-45 deg, nsteps time steps over 14 days), step s seen
    by frame floor(s K / nsteps); detector annulus 1.4-4 R_sun kept; unit
    sphere masked; frame f is the base phantom rotated 0.5 deg * f."""
    nn, lo, hi = box(n, 4.0)
    lons, frames = [], []
    for s in range(nsteps):
        day = 14.0 * s / nsteps
        for sign in (1.0, -1.0):
            lons.append(sign * 45.0 - ROT_DEG_PER_DAY * day)
            frames.append(s * K // nsteps)
    views, pix = make_views(lons, (npix, npix), 8.0)
    mm = sphere_map_mask(nn, lo, hi)
    dm = annulus_data_mask(views, pix, 1.4, 4.0)
    blobs = draw_shell_blobs(np.random.default_rng(3), 16)
    rad = radial_cube(nn, lo, hi)
    x = np.stack([(blob_cube(nn, lo, hi, blobs, 0.5 * f) + rad) * mm for f in range(K)])
    g = Geometry(nn, lo, hi, views, pix, np.array(frames, dtype=np.int32), K, dm, mm)
    return Workload(f"cor1-{K}x{n}^3-{len(lons)}x{npix}^2", g, x, 1e-2, 10.0, 0)


def cor1_extras() -> list:
    """Four independent reconstructions of uneven sizes batched with the
    time-evolving model."""
    out = []
    for i, n in enumerate((64, 96, 128, 192)):
        nn, lo, hi = box(n, 1.5)
        views, pix = make_views([22.5 * k for k in range(16)], (256, 256), 3.4)
        x = blob_cube(nn, lo, hi, draw_blobs(np.random.default_rng(300 + i), 16))
        out.append(Workload(f"extra-{n}^3", Geometry(nn, lo, hi, views, pix), x, 1e-2))
    return out


# ------------------------------------------ the paper's projector scaling sweeps


SWEEP_IMAGE_SIDES = (128, 256, 512, 1024)  # 64 views, 128^3 cube (Sec. "Performance", image-size table)
SWEEP_CUBE_SIDES = (128, 256, 512, 1024)  # 64 views of 256^2 (Sec. "Performance", cube-size table)


def sweep_geometry(n: int = 128, npix: int = 256, nviews: int = 64) -> Geometry:
    """The projector benchmark set-up of the paper's Performance section: an
    n^3 cube (here on [-1.5, 1.5]^3 R_sun) and `nviews` images of npix^2,
    no mask and no obstacle.  The paper gives no pointing; the views here sit
    at 215 R_sun, equally spaced in longitude around the equator starting half
    a step from longitude 0 (no observer on an axis or a diagonal of the grid,
    whose rays would run exactly along voxel edges), FOV 3.2."""
    nn, lo, hi = box(n, 1.5)
    step = 360.0 / nviews
    views, pix = make_views(0.5 * step + step * np.arange(nviews), (npix, npix), 3.2)
    return Geometry(nn, lo, hi, views, pix)


def sweep_cube_parts(n: int, seed: int = 11) -> tuple:
    """Three seeded float32 vectors (a over x, b over y, c over z) of the
    separable sweep phantom x[k, j, i] = (c[k] + b[j]) + a[i], values in
    [0.5, 1.5]: cheap to hold at 1024^3 and to evaluate at single voxels."""
    rng = np.random.default_rng(seed)
    a, b, c = (rng.uniform(1.0 / 6.0, 0.5, size=n).astype(np.float32) for _ in range(3))
    return a, b, c


def sweep_cube(parts) -> np.ndarray:
    """The whole sweep phantom, float32 (nz, ny, nx), summed in float32 as
    (c + b) + a."""
    a, b, c = parts
    return (c[:, None, None] + b[None, :, None]) + a[None, None, :]


def sweep_values(parts, flat_idx) -> np.ndarray:
    """The sweep phantom at flat voxel indices (k n + j) n + i, float32
    arithmetic in the same order as sweep_cube."""
    a, b, c = parts
    n = a.size
    idx = np.asarray(flat_idx, dtype=np.int64)
    i, j, k = idx % n, (idx // n) % n, idx // (n * n)
    return (c[k] + b[j]) + a[i]
