"""FP64 CPU oracle for the TomograPy hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library (``paper_1103_5904_amd``) and never imports it.

Contents, each following the paper (Barbey, Guennou & Auchere, Solar Physics,
"TomograPy: a fast, instrument-independent, solar tomography software"):

* ``project`` / ``backproject``: the line-of-sight projector of Eq. lo and its
  transpose, by Siddon's merge of plane-crossing sets (C core in
  ``oracle.c``); ``ray_row_bruteforce`` recomputes one row straight from the
  definition (per-voxel slab clip).
* ``laplacian6`` / ``laplacian_t``: D^T D for the finite-difference priors
  (Sec. "Single Spacecraft Static Tomography"; Eq. stsrt for time);
  ``voxel_heights`` / ``height_prior``: R D^T D R, the prior weighted by
  voxel height of Eq. srt_inversion.
* ``ray_gains``: the per-instrument gains of Eq. two_spacecraft /
  Eq. lin2space, applied by ``project`` and ``backproject`` when the
  geometry carries them.
* ``normal_operator`` / ``cg``: the normal equations of Eq. criterion,
  (P^T P + lambda D^T D) x = P^T y, solved by textbook conjugate gradient.
* ``fcg``, ``convnet_*``, ``adam_step``: the preconditioner the paper names
  as untried (Sec. "Smooth Temporal Evolution"), as flexible CG around a small
  3-D convolution network, and the network's training step.
* ``view_from_wcs``: the oracle's own reading of WCS pointing keywords.
* ``thomson_*``: the white-light Thomson-scattering operators of
  Sec. "White Light: Thomson Scattering" (Eq. thomson_lo, Eq. brightness,
  Eq. thomson_direct): pB = O P M n_e and B = (-O P M + P M') n_e.

Parity status: every function above is pinned by ``tests/test_oracle_*.py``
except the learned network's *benefit*, which the paper does not quantify
(parity unpinned; only its arithmetic is pinned).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C core with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        _lib.ora_count_crossings.restype = ctypes.c_int64
        _lib.ora_max_threads.restype = ctypes.c_int
    return _lib


def max_threads() -> int:
    return int(_load().ora_max_threads())


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _geom_args(g):
    n = np.ascontiguousarray(g.n, dtype=np.int32)
    lo = np.ascontiguousarray(g.lo, dtype=np.float64)
    hi = np.ascontiguousarray(g.hi, dtype=np.float64)
    views = np.ascontiguousarray(g.views, dtype=np.float64)
    npix = np.ascontiguousarray(g.npix, dtype=np.int32)
    vf = None if g.view_frame is None else np.ascontiguousarray(g.view_frame, dtype=np.int32)
    dm = None if g.data_mask is None else np.ascontiguousarray(g.data_mask, dtype=np.uint8)
    mm = None if g.map_mask is None else np.ascontiguousarray(g.map_mask, dtype=np.uint8)
    return n, lo, hi, views, npix, vf, dm, mm


def _obstacle(g):
    """The geometry's opaque sphere as (cx, cy, cz, R) float64, or None."""
    ob = getattr(g, "obstacle", None)
    return None if ob is None else np.ascontiguousarray(ob, dtype=np.float64).reshape(4)


def ray_gains(g):
    """The gain of each ray's instrument (Eq. two_spacecraft, Eq. lin2space:
    view v's rows of the stacked operator are g_v P_v), one value per pixel
    in image order, or None when the geometry has no gains (all 1)."""
    gn = getattr(g, "gains", None)
    if gn is None:
        return None
    gn = np.asarray(gn, dtype=np.float64).reshape(g.nviews)
    return np.repeat(gn, g.npix[:, 0].astype(np.int64) * g.npix[:, 1])


# ------------------------------------------------------------- projector


def project(g, cube, nthreads: int = 0, use_map_mask: bool = True) -> np.ndarray:
    """(G P M x): one line integral per pixel, concatenated over views, times
    the gain of the view's instrument when the geometry has gains (G, the
    diagonal of ``ray_gains``)."""
    lib = _load()
    n, lo, hi, views, npix, vf, dm, mm = _geom_args(g)
    x = np.ascontiguousarray(cube, dtype=np.float64)
    assert x.size == g.nvox * g.nframes
    out = np.empty(g.nrays, dtype=np.float64)
    rc = lib.ora_project(_p(n), _p(lo), _p(hi), ctypes.c_int(g.nviews), _p(views), _p(npix),
                         _p(vf), _p(dm), _p(mm if use_map_mask else None), _p(_obstacle(g)), _p(x),
                         _p(out), ctypes.c_int(nthreads))
    if rc:
        raise MemoryError("oracle projection failed")
    gr = ray_gains(g)
    return out if gr is None else out * gr


def backproject(g, images, nthreads: int = 0, use_map_mask: bool = True) -> np.ndarray:
    """(M P^T G y), the transpose of ``project``, returned in the geometry's
    cube shape."""
    lib = _load()
    n, lo, hi, views, npix, vf, dm, mm = _geom_args(g)
    y = np.ascontiguousarray(images, dtype=np.float64).ravel()
    assert y.size == g.nrays
    gr = ray_gains(g)
    if gr is not None:
        y = np.ascontiguousarray(y * gr)
    out = np.empty(g.nvox * g.nframes, dtype=np.float64)
    rc = lib.ora_backproject(_p(n), _p(lo), _p(hi), ctypes.c_int(g.nviews), _p(views), _p(npix),
                             _p(vf), ctypes.c_int(g.nframes), _p(dm),
                             _p(mm if use_map_mask else None), _p(_obstacle(g)), _p(y), _p(out),
                             ctypes.c_int(0), ctypes.c_int(nthreads))
    if rc:
        raise MemoryError("oracle back-projection failed")
    return out.reshape(g.cube_shape())


def count_crossings(g, nthreads: int = 0) -> int:
    """Positive-length ray/voxel segments summed over all unmasked rays."""
    lib = _load()
    n, lo, hi, views, npix, _, dm, _ = _geom_args(g)
    c = lib.ora_count_crossings(_p(n), _p(lo), _p(hi), ctypes.c_int(g.nviews), _p(views),
                                _p(npix), _p(dm), _p(_obstacle(g)), ctypes.c_int(nthreads))
    if c < 0:
        raise MemoryError("oracle count failed")
    return int(c)


def trace_ray(n, lo, hi, o, d, obstacle=None):
    """Siddon segments of the half-line o + t d: (voxel index, length, t at
    the segment's entry), in order along the ray, up to the first contact
    with the obstacle sphere (cx, cy, cz, R) when one is given."""
    lib = _load()
    n = np.ascontiguousarray(n, dtype=np.int32)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    cap = int(n.sum()) + 3
    idx = np.empty(cap, dtype=np.int32)
    ln = np.empty(cap, dtype=np.float64)
    tl = np.empty(cap, dtype=np.float64)
    ob = None if obstacle is None else np.ascontiguousarray(obstacle, dtype=np.float64).reshape(4)
    k = lib.ora_trace_ray(_p(n), _p(lo), _p(hi), _p(o), _p(d), _p(ob), _p(idx), _p(ln), _p(tl),
                          ctypes.c_int(cap))
    if k < 0:
        raise RuntimeError("segment buffer overflow")
    return idx[:k].copy(), ln[:k].copy(), tl[:k].copy()


def ray_row_bruteforce(n, lo, hi, o, d, obstacle=None) -> np.ndarray:
    """Row of P for one ray from the plain definition: one slab clip per voxel
    (each voxel's interval cut at the obstacle's first contact, if any)."""
    lib = _load()
    n = np.ascontiguousarray(n, dtype=np.int32)
    out = np.empty(int(np.prod(n)), dtype=np.float64)
    ob = None if obstacle is None else np.ascontiguousarray(obstacle, dtype=np.float64).reshape(4)
    lib.ora_ray_row_bruteforce(_p(n), _p(np.ascontiguousarray(lo, dtype=np.float64)),
                               _p(np.ascontiguousarray(hi, dtype=np.float64)),
                               _p(np.ascontiguousarray(o, dtype=np.float64)),
                               _p(np.ascontiguousarray(d, dtype=np.float64)), _p(ob), _p(out))
    return out


def pixel_direction(view16, npix, col, row) -> np.ndarray:
    lib = _load()
    v = np.ascontiguousarray(view16, dtype=np.float64)
    p = np.ascontiguousarray(npix, dtype=np.int32)
    d = np.empty(3)
    lib.ora_pixel_direction(_p(v), _p(p), ctypes.c_int(col), ctypes.c_int(row), _p(d))
    return d


def dense_matrix(g) -> np.ndarray:
    """The geometric P as a dense (rays x voxels) matrix, one Siddon trace
    per ray (tiny geometries only; gains are not applied).  Data-masked rows
    are zero."""
    rows = []
    off = g.view_offsets()
    for v in range(g.nviews):
        ncol, nrow = (int(t) for t in g.npix[v])
        for r in range(ncol * nrow):
            row = np.zeros(g.nvox)
            if g.data_mask is None or g.data_mask[off[v] + r]:
                d = pixel_direction(g.views[v], g.npix[v], r % ncol, r // ncol)
                idx, ln, _ = trace_ray(g.n, g.lo, g.hi, g.views[v][0:3], d)
                np.add.at(row, idx, ln)
            rows.append(row)
    return np.array(rows)


# --------------------------------------------------------------- priors


def _dtd_along(x, axis):
    """D^T D x for the forward difference along one axis, between in-range
    neighbours only (free ends)."""
    dx = np.diff(x, axis=axis)  # (D x)_k = x_{k+1} - x_k
    out = np.zeros_like(x)
    sl = [slice(None)] * x.ndim
    # D^T d: component k receives -d_k (as the left end of pair k) and
    # +d_{k-1} (as the right end of pair k-1).
    sl[axis] = slice(0, -1)
    out[tuple(sl)] -= dx
    sl[axis] = slice(1, None)
    out[tuple(sl)] += dx
    return out


def laplacian6(x) -> np.ndarray:
    """D^T D with D the forward differences along x, y and z of each voxel
    cube (the last three axes), i.e. the Neumann 6-neighbour graph Laplacian."""
    x = np.asarray(x, dtype=np.float64)
    return sum(_dtd_along(x, ax) for ax in (-1, -2, -3))


def laplacian_t(x) -> np.ndarray:
    """D_t^T D_t with D_t the forward difference between consecutive time
    frames (axis 0 of a (frames, nz, ny, nx) array)."""
    x = np.asarray(x, dtype=np.float64)
    if x.shape[0] < 2:
        return np.zeros_like(x)
    return _dtd_along(x, 0)


def voxel_heights(g, height):
    """Diagonal of R in Eq. srt_inversion for height = (cx, cy, cz, offset):
    the distance from each voxel's centre to the point (cx, cy, cz) (the
    Sun's centre), plus offset, in box units, shaped (nz, ny, nx)."""
    cx, cy, cz, off = (float(t) for t in height)
    ax = []
    for a, c in zip(range(3), (cx, cy, cz)):
        n = int(g.n[a])
        step = (float(g.hi[a]) - float(g.lo[a])) / n
        ax.append(float(g.lo[a]) + (np.arange(n) + 0.5) * step - c)
    zz, yy, xx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.sqrt(xx * xx + yy * yy + zz * zz) + off


def height_prior(x, h) -> np.ndarray:
    """R D^T D R x with R = diag(h) (Eq. srt_inversion): the spatial prior
    of every frame with each voxel weighted by its height."""
    x = np.asarray(x, dtype=np.float64)
    return h * laplacian6(h * x)


def normal_operator(g, lam_r, lam_t=0.0, nthreads=0, height=None):
    """x -> M (P^T G^2 P + lam_r R D^T D R + lam_t D_t^T D_t) M x on the
    geometry's cube shape: the map mask M restricts the unknowns (operator
    P M), G holds the instruments' gains (Eq. srt_multiple_inv) and R the
    voxel heights when ``height`` = (cx, cy, cz, offset) is given
    (Eq. srt_inversion; R = I otherwise)."""
    mm = None if g.map_mask is None else g.map_mask.astype(np.float64)
    h = None if height is None else voxel_heights(g, height)

    def apply(x):
        x = np.asarray(x, dtype=np.float64).reshape(g.cube_shape())
        xm = x * mm if mm is not None else x
        q = backproject(g, project(g, xm, nthreads), nthreads, use_map_mask=False)
        q = q + lam_r * (laplacian6(xm) if h is None else height_prior(xm, h))
        if lam_t:
            q = q + lam_t * laplacian_t(xm)
        return q * mm if mm is not None else q

    return apply


def rhs(g, y, nthreads=0):
    """b = M P^T G y."""
    return backproject(g, y, nthreads)


def criterion(g, x, y, lam_r, lam_t=0.0, height=None):
    """J(x) = ||y - G P M x||^2 + lam_r ||D R M x||^2 + lam_t ||D_t M x||^2
    (Eq. criterion, Eq. stsrt, Eq. srt_inversion, Eq. srt_multiple_inv;
    R = I without ``height``)."""
    x = np.asarray(x, dtype=np.float64).reshape(g.cube_shape())
    xm = x * g.map_mask if g.map_mask is not None else x
    res = y - project(g, xm)
    j = float(res @ res)
    rx = xm if height is None else xm * voxel_heights(g, height)
    for ax in (-1, -2, -3):
        j += lam_r * float(np.sum(np.diff(rx, axis=ax) ** 2))
    if lam_t and xm.ndim == 4:
        j += lam_t * float(np.sum(np.diff(xm, axis=0) ** 2))
    return j


# --------------------------------------------------------------- solvers


def cg(apply_a, b, x0=None, n_iter=50, rtol=0.0, record=False):
    """Textbook conjugate gradient on A x = b (A symmetric positive
    definite), FP64 throughout.  Stops after n_iter iterations or when
    ||r_k|| <= rtol ||b||.  Returns (x, history of ||r_k||/||b||[, iterates])."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_a(x) if x0 is not None else b.copy()
    p = r.copy()
    rr = float(np.vdot(r, r))
    bn = float(np.sqrt(np.vdot(b, b)))
    hist = [np.sqrt(rr) / bn]
    iters = [x.copy()] if record else None
    for _ in range(n_iter):
        if rtol and hist[-1] <= rtol:
            break
        q = apply_a(p)
        alpha = rr / float(np.vdot(p, q))
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(np.vdot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        hist.append(np.sqrt(rr) / bn)
        if record:
            iters.append(x.copy())
    return (x, np.array(hist), iters) if record else (x, np.array(hist))


def fcg(apply_a, b, precond, x0=None, n_iter=50, rtol=0.0, window=3, min_drop=1e-6):
    """Flexible CG with a (possibly non-linear) preconditioner z = N(r) and
    the Polak-Ribiere choice beta = z_{k+1}.(r_{k+1} - r_k) / z_k.r_k.

    Fall-back to plain CG, restarted from the current iterate, when either
    (a) the residual norm has failed to fall by more than a relative
    ``min_drop`` for ``window`` consecutive iterations, or (b) z.r is not
    positive or not finite (the preconditioned residual is not a descent
    direction).  Returns (x, relative-residual history, iteration of the
    fall-back or -1)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_a(x) if x0 is not None else b.copy()
    bn = float(np.sqrt(np.vdot(b, b)))
    hist = [float(np.sqrt(np.vdot(r, r))) / bn]
    use_net, fell_back, stall = True, -1, 0
    z = precond(r)
    zr = float(np.vdot(z, r))
    if not (np.isfinite(zr) and zr > 0.0):
        use_net, fell_back = False, 0
        z, zr = r.copy(), float(np.vdot(r, r))
    p = z.copy()
    for k in range(n_iter):
        if rtol and hist[-1] <= rtol:
            break
        q = apply_a(p)
        alpha = zr / float(np.vdot(p, q))
        x = x + alpha * p
        r_new = r - alpha * q
        hist.append(float(np.sqrt(np.vdot(r_new, r_new))) / bn)
        stall = stall + 1 if hist[-1] > (1.0 - min_drop) * hist[-2] else 0
        z_new = None
        if use_net and stall < window:
            z_new = precond(r_new)
            zr_new = float(np.vdot(z_new, r_new))
            if not (np.isfinite(zr_new) and zr_new > 0.0):
                z_new = None
        if use_net and z_new is None:  # restart as plain CG
            use_net, fell_back, stall = False, k + 1, 0
            r = r_new
            z, zr = r.copy(), float(np.vdot(r, r))
            p = z.copy()
            continue
        if use_net:
            beta = float(np.vdot(z_new, r_new - r)) / zr
        else:  # plain CG
            z_new = r_new.copy()
            zr_new = float(np.vdot(r_new, r_new))
            beta = zr_new / zr
        p = z_new + beta * p
        r, z, zr = r_new, z_new, zr_new
    return x, np.array(hist), fell_back


# ----------------------------------------------------- convolution network

CHANNELS = (1, 16, 16, 1)


def conv3d(x, w, b=None):
    """3x3x3 convolution, zero padding 1; x: (cin, nz, ny, nx), w: (cout,
    cin, 3, 3, 3)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    cout, cin = w.shape[0], w.shape[1]
    nz, ny, nx = x.shape[1:]
    out = np.empty((cout, nz, ny, nx))
    bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
    lib.ora_conv3d_forward(cin, cout, nz, ny, nx, _p(x), _p(w), _p(bb), _p(out))
    return out


def conv3d_backward(x, w, gout):
    """Gradients (d input, d weight, d bias) of a conv3d given d output."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    gout = np.ascontiguousarray(gout, dtype=np.float64)
    cout, cin = w.shape[0], w.shape[1]
    nz, ny, nx = x.shape[1:]
    gin = np.empty_like(x)
    gw = np.empty_like(w)
    gb = np.empty(cout)
    lib.ora_conv3d_backward_data(cin, cout, nz, ny, nx, _p(gout), _p(w), _p(gin))
    lib.ora_conv3d_backward_weight(cin, cout, nz, ny, nx, _p(x), _p(gout), _p(gw), _p(gb))
    return gin, gw, gb


def convnet_forward(params, r, keep=False):
    """N(r) = conv3(ReLU(conv2(ReLU(conv1(r))))); params = [w1, b1, w2, b2,
    w3, b3]; r: (nz, ny, nx).  With keep=True also returns the activations."""
    w1, b1, w2, b2, w3, b3 = params
    a0 = np.asarray(r, dtype=np.float64)[None]
    h1 = conv3d(a0, w1, b1)
    a1 = np.maximum(h1, 0.0)
    h2 = conv3d(a1, w2, b2)
    a2 = np.maximum(h2, 0.0)
    out = conv3d(a2, w3, b3)[0]
    return (out, (a0, h1, a1, h2, a2)) if keep else out


def convnet_backward(params, acts, gout):
    """Parameter gradients of N at the stored activations, for d loss / d
    output = gout (nz, ny, nx)."""
    w1, b1, w2, b2, w3, b3 = params
    a0, h1, a1, h2, a2 = acts
    g2, gw3, gb3 = conv3d_backward(a2, w3, np.asarray(gout, dtype=np.float64)[None])
    g2 = g2 * (h2 > 0)
    g1, gw2, gb2 = conv3d_backward(a1, w2, g2)
    g1 = g1 * (h1 > 0)
    _, gw1, gb1 = conv3d_backward(a0, w1, g1)
    return [gw1, gb1, gw2, gb2, gw3, gb3]


def mse_loss_and_grad(params, r, target):
    """Loss = mean((N(r) - target)^2) and its parameter gradients."""
    out, acts = convnet_forward(params, r, keep=True)
    diff = out - target
    loss = float(np.mean(diff * diff))
    grads = convnet_backward(params, acts, 2.0 * diff / diff.size)
    return loss, grads


def normalized_precond(params):
    """z = ||r|| N(r / ||r||): the network sees unit-norm residuals, as in its
    training pairs."""

    def apply(r):
        s = float(np.sqrt(np.vdot(r, r)))
        if s == 0.0:
            return np.zeros_like(r)
        return s * convnet_forward(params, r / s)

    return apply


def linear_filter_net(h):
    """Weights for which N(r) = h * r exactly, for any 3x3x3 filter h
    (cross-correlation, zero padding).  conv1 splits r into (r, -r) and the
    ReLU keeps r+ and r-; conv2 applies h+ and h- (the positive and negative
    parts of h) to each, giving four non-negative channels that the second
    ReLU leaves alone; conv3 recombines them:
    h*r = h+*r+ - h-*r+ - h+*r- + h-*r-."""
    h = np.asarray(h, dtype=np.float64).reshape(3, 3, 3)
    hp, hm = np.maximum(h, 0.0), np.maximum(-h, 0.0)
    w1 = np.zeros((16, 1, 3, 3, 3))
    w1[0, 0, 1, 1, 1], w1[1, 0, 1, 1, 1] = 1.0, -1.0
    w2 = np.zeros((16, 16, 3, 3, 3))
    w2[0, 0], w2[1, 0], w2[2, 1], w2[3, 1] = hp, hm, hp, hm
    w3 = np.zeros((1, 16, 3, 3, 3))
    w3[0, 0:4, 1, 1, 1] = [1.0, -1.0, -1.0, 1.0]
    return [w1, np.zeros(16), w2, np.zeros(16), w3, np.zeros(1)]


def identity_net(scale=1.0):
    """Weights for which N(r) = scale * r exactly."""
    h = np.zeros((3, 3, 3))
    h[1, 1, 1] = scale
    return linear_filter_net(h)


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), in place; t counts from 1."""
    for p, g, mi, vi in zip(params, grads, m, v):
        mi *= b1
        mi += (1.0 - b1) * g
        vi *= b2
        vi += (1.0 - b2) * g * g
        mhat = mi / (1.0 - b1 ** t)
        vhat = vi / (1.0 - b2 ** t)
        p -= lr * mhat / (np.sqrt(vhat) + eps)


# ------------------------------------------------------------------- WCS


def view_from_wcs(dsun, hgln_deg, hglt_deg, crval1_as, crval2_as, crota_deg,
                  cdelt1_as, cdelt2_as, crpix1, crpix2, ncol, nrow):
    """View row (16 numbers) and (ncol, nrow) from helioprojective TAN WCS
    keywords: observer at distance dsun (R_sun) and heliographic longitude /
    latitude; reference direction (crval1, crval2) arcsec west / north of Sun
    centre; crota the image rotation; cdelt in arcsec per pixel; crpix
    1-based (FITS)."""
    a2r = np.pi / (180.0 * 3600.0)
    lon, lat = np.deg2rad(hgln_deg), np.deg2rad(hglt_deg)
    obs = dsun * np.array([np.cos(lat) * np.cos(lon), np.cos(lat) * np.sin(lon), np.sin(lat)])
    # observer's Sun-centred frame: toward Sun centre, solar west, solar north
    to_sun = -obs / np.linalg.norm(obs)
    north = np.array([0.0, 0.0, 1.0]) - to_sun[2] * to_sun
    north /= np.linalg.norm(north)
    west = np.cross(to_sun, north)
    tx, ty = crval1_as * a2r, crval2_as * a2r
    # direction of the reference point and the unit tangents along +theta_y
    # (meridian through it) and +theta_x
    w = np.cos(ty) * np.cos(tx) * to_sun + np.cos(ty) * np.sin(tx) * west + np.sin(ty) * north
    e_ty = -np.sin(ty) * np.cos(tx) * to_sun - np.sin(ty) * np.sin(tx) * west + np.cos(ty) * north
    e_tx = np.cross(w, e_ty)
    rho = np.deg2rad(crota_deg)
    u = np.cos(rho) * e_tx + np.sin(rho) * e_ty
    v = -np.sin(rho) * e_tx + np.cos(rho) * e_ty
    row = np.concatenate([obs, w, u, v, [cdelt1_as * a2r, cdelt2_as * a2r],
                          [crpix1 - 1.0, crpix2 - 1.0]])
    return row, np.array([ncol, nrow], dtype=np.int32)


# ------------------------------------------------------- Thomson scattering


def thomson_c1234(sin_omega):
    """Billings' coefficients C1..C4 of Eq. 4C at sin(Omega) = R_sun / r,
    Omega the half-angle of the solar disc seen from the scattering point.
    C4 takes +1/8 in front of its bracket: the printed minus sign would make
    the fully limb-darkened total brightness negative, and only +1/8 gives
    C4 / C3 -> 2/3 as Omega -> 0 (the flux of a linearly limb-darkened disc
    relative to a uniform one), as C2 / C1 does."""
    s = np.asarray(sin_omega, dtype=np.float64)
    c = np.sqrt(1.0 - s * s)
    lg = np.log((1.0 + s) / c)
    c1 = c * s * s
    c2 = -0.125 * (1.0 - 3.0 * s * s - (c * c / s) * (1.0 + 3.0 * s * s) * lg)
    c3 = 4.0 / 3.0 - c - c ** 3 / 3.0
    c4 = 0.125 * (5.0 + s * s - (c * c / s) * (5.0 - s * s) * lg)
    return c1, c2, c3, c4


def thomson_voxel_weights(g, u, sun=(0.0, 0.0, 0.0, 1.0)):
    """Per-voxel diagonals m_j and m'_j (Eq. thomson_lo, with the limb-
    darkening factor u on C2 and C4 and the factor 2 of the radial term
    taken from Eq. brightness): at the voxel centre's distance r from the
    Sun's centre, in solar radii R (sun = (cx, cy, cz, R)),
      m  = ((1 - u) C1 + u C2) / r^4,   m' = 2 ((1 - u) C3 + u C4) / r^2,
    and 0 for centres on or inside the photosphere (r <= 1).  Shape of one
    frame, z slowest."""
    nx, ny, nz = g.n
    cen = [g.lo[a] + (np.arange(k) + 0.5) * (g.hi[a] - g.lo[a]) / k for a, k in enumerate((nx, ny, nz))]
    zz, yy, xx = np.meshgrid(cen[2], cen[1], cen[0], indexing="ij")
    r = np.sqrt((xx - sun[0]) ** 2 + (yy - sun[1]) ** 2 + (zz - sun[2]) ** 2) / sun[3]
    out = r > 1.0
    rr = np.where(out, r, 2.0)
    c1, c2, c3, c4 = thomson_c1234(1.0 / rr)
    m = np.where(out, ((1.0 - u) * c1 + u * c2) / rr ** 4, 0.0)
    mp = np.where(out, 2.0 * ((1.0 - u) * c3 + u * c4) / rr ** 2, 0.0)
    return m, mp


def thomson_pixel_weights(g, sun=(0.0, 0.0, 0.0, 1.0)):
    """o_k = rho_k^2 (Eq. thomson_lo): the squared impact parameter, in solar
    radii, of every pixel's line of sight (its distance from the Sun's
    centre), views concatenated."""
    out = np.empty(g.nrays)
    off = g.view_offsets()
    c = np.asarray(sun[:3], dtype=np.float64)
    for v in range(g.nviews):
        ncol, nrow = (int(k) for k in g.npix[v])
        o = g.views[v, 0:3] - c
        k = off[v]
        for row in range(nrow):
            for col in range(ncol):
                d = pixel_direction(g.views[v], g.npix[v], col, row)
                cr = np.cross(o, d)
                out[k] = (cr @ cr) / (d @ d) / sun[3] ** 2
                k += 1
    return out


def _frames(w, g):
    return w if g.nframes == 1 else np.broadcast_to(w, (g.nframes,) + w.shape)


def thomson_project(g, ne, u, kind, scale=1.0, sun=(0.0, 0.0, 0.0, 1.0)):
    """Eq. thomson_direct without noise: kind 'pB' gives scale O P M n_e,
    kind 'B' gives scale (-O P M + P M') n_e."""
    m, mp = thomson_voxel_weights(g, u, sun)
    o = thomson_pixel_weights(g, sun)
    ne = np.asarray(ne, dtype=np.float64)
    pm = project(g, ne * _frames(m, g))
    if kind == "pB":
        return scale * o * pm
    return scale * (project(g, ne * _frames(mp, g)) - o * pm)


def thomson_backproject(g, y, u, kind, scale=1.0, sun=(0.0, 0.0, 0.0, 1.0)):
    """Transposes: scale M P^T O y (pB), scale (M' P^T y - M P^T O y) (B)."""
    m, mp = thomson_voxel_weights(g, u, sun)
    o = thomson_pixel_weights(g, sun)
    y = np.asarray(y, dtype=np.float64).ravel()
    bo = backproject(g, o * y) * _frames(m, g)
    if kind == "pB":
        return scale * bo
    return scale * (backproject(g, y) * _frames(mp, g) - bo)

