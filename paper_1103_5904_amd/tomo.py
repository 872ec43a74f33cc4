"""ctypes binding of libtomo (include/tomo.h): argument marshalling only.

Every numeric step runs in the HIP library; PyTorch supplies device memory
and the current stream.  If libtomo.so has not been built, importing the
functions works but every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_void_p

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtomo.so")

TOMO_OK = 0
TOMO_EINVAL = -1
TOMO_EHIP = -2
TOMO_ENONFINITE = -3
TOMO_ENOCONV = -4
TOMO_ENOMEM = -5
TOMO_EUNSUPPORTED = -6

BP_AUTO, BP_ATOMIC, BP_BINNED, BP_BLOCKED = 0, 1, 2, 3


class TomoError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"libtomo status {status}: {message}")
        self.status = status


class TomoCube(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("nframes", c_int32),
                ("box_min", c_double * 3), ("box_max", c_double * 3)]


class TomoView(ctypes.Structure):
    _fields_ = [("obs", c_double * 3), ("w", c_double * 3), ("u", c_double * 3),
                ("v", c_double * 3), ("cdelt", c_double * 2), ("crpix", c_double * 2),
                ("ncol", c_int32), ("nrow", c_int32), ("frame", c_int32), ("reserved", c_int32)]


class TomoObstacle(ctypes.Structure):
    _fields_ = [("center", c_double * 3), ("radius", c_double)]


class TomoGeometry(ctypes.Structure):
    _fields_ = [("cube", TomoCube), ("nviews", c_int32), ("reserved", c_int32),
                ("views", POINTER(TomoView)), ("data_mask", c_void_p), ("map_mask", c_void_p),
                ("obstacle", POINTER(TomoObstacle)), ("gains", POINTER(c_double))]


class TomoHeight(ctypes.Structure):
    _fields_ = [("center", c_double * 3), ("offset", c_double)]


class ThomsonParams(ctypes.Structure):
    _fields_ = [("u", c_double), ("scale", c_double), ("sun_center", c_double * 3), ("sun_radius", c_double)]


THOMSON_KINDS = {"pB": 0, "B": 1}


class Tuning(ctypes.Structure):
    _fields_ = [("p_bundle", c_int32), ("p_xcd_remap", c_int32), ("bp_bundle", c_int32),
                ("bp_xcd_remap", c_int32), ("bp_lds_bins", c_int32), ("bp_default", c_int32),
                ("bp_block", c_int32 * 3), ("bp_splits", c_int32), ("bp_threads", c_int32),
                ("p_layout", c_int32), ("bp_ray_table", c_int32)]


class CgParams(ctypes.Structure):
    _fields_ = [("lambda_r", c_double), ("lambda_t", c_double), ("max_iter", c_int32),
                ("x0_given", c_int32), ("rtol", c_double), ("check_every", c_int32),
                ("use_graph", c_int32), ("precond", c_void_p), ("fallback_window", c_int32),
                ("bp_strategy", c_int32), ("min_drop", c_double), ("record_x", c_void_p),
                ("record_r", c_void_p), ("record_count", c_int32), ("reserved", c_int32),
                ("height", POINTER(TomoHeight)), ("workspace", c_void_p), ("workspace_bytes", ctypes.c_size_t)]


class CgReport(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("status", c_int32), ("fell_back", c_int32),
                ("n_project", c_int32), ("n_backproject", c_int32), ("reserved", c_int32),
                ("rel_res", c_double), ("true_rel_res", c_double), ("bnorm", c_double),
                ("ms_project", c_double), ("ms_backproject", c_double),
                ("history", POINTER(c_double)), ("history_cap", c_int32),
                ("history_len", c_int32), ("time_kernels", c_int32), ("reserved2", c_int32)]


EXPORTS = [
    "tomo_project", "tomo_backproject", "tomo_backproject_ex", "tomo_count_crossings",
    "tomo_thomson_project", "tomo_thomson_backproject",
    "tomo_trace_ray", "tomo_apply_prior", "tomo_apply_height_prior", "tomo_cg_solve", "tomo_cg_default_params",
    "tomo_view_from_wcs", "tomo_validate_geometry", "tomo_geometry_pixels",
    "tomo_release_cache", "tomo_status_string", "tomo_last_error", "tomo_binning_spills",
    "tomo_get_tuning", "tomo_set_tuning", "tomo_convnet_workspace_bytes", "tomo_convnet_forward",
    "tomo_convnet_loss_grad", "tomo_convnet_backward", "tomo_adam_step", "tomo_autotune",
    "tomo_get_class_tuning", "tomo_autotune_clear", "tomo_batch_create", "tomo_batch_destroy",
    "tomo_batch_project", "tomo_batch_backproject", "tomo_batch_binning_spills", "tomo_batch_items",
    "tomo_batch_cg_solve", "tomo_backproject_noalloc", "tomo_autotune_data", "tomo_cg_workspace_bytes",
]
NPARAMS = 7809

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.tomo_status_string.restype = ctypes.c_char_p
        L.tomo_last_error.restype = ctypes.c_char_p
        L.tomo_geometry_pixels.restype = c_int64
        L.tomo_project.argtypes = [POINTER(TomoGeometry), c_void_p, c_void_p, c_void_p]
        L.tomo_backproject.argtypes = [POINTER(TomoGeometry), c_void_p, c_void_p, ctypes.c_int,
                                       c_void_p]
        L.tomo_backproject_ex.argtypes = [POINTER(TomoGeometry), c_void_p, c_void_p, ctypes.c_int,
                                          ctypes.c_int, c_void_p]
        L.tomo_backproject_noalloc.argtypes = [POINTER(TomoGeometry), c_void_p, c_void_p, ctypes.c_int,
                                               c_void_p]
        L.tomo_count_crossings.argtypes = [POINTER(TomoGeometry), POINTER(c_int64), c_void_p]
        L.tomo_trace_ray.argtypes = [POINTER(TomoGeometry), c_int32, c_int32, c_int32,
                                     POINTER(c_int32), POINTER(c_double), POINTER(c_double),
                                     c_int32, POINTER(c_int32)]
        L.tomo_apply_prior.argtypes = [POINTER(TomoCube), c_double, c_double, c_void_p, c_void_p,
                                       ctypes.c_int, c_void_p]
        L.tomo_apply_height_prior.argtypes = [POINTER(TomoCube), POINTER(TomoHeight), c_double, c_double,
                                              c_void_p, c_void_p, ctypes.c_int, c_void_p]
        L.tomo_cg_solve.argtypes = [POINTER(TomoGeometry), c_void_p, c_void_p, POINTER(CgParams),
                                    POINTER(CgReport), c_void_p]
        L.tomo_cg_default_params.argtypes = [POINTER(CgParams)]
        L.tomo_cg_workspace_bytes.argtypes = [POINTER(TomoGeometry), POINTER(CgParams)]
        L.tomo_cg_workspace_bytes.restype = ctypes.c_size_t
        L.tomo_view_from_wcs.argtypes = [c_double] * 10 + [c_int32, c_int32, POINTER(TomoView)]
        L.tomo_validate_geometry.argtypes = [POINTER(TomoGeometry)]
        L.tomo_binning_spills.argtypes = [POINTER(TomoGeometry), POINTER(c_int64)]
        L.tomo_get_tuning.argtypes = [POINTER(Tuning)]
        L.tomo_convnet_workspace_bytes.argtypes = [POINTER(TomoCube)]
        L.tomo_convnet_workspace_bytes.restype = ctypes.c_size_t
        L.tomo_convnet_forward.argtypes = [POINTER(TomoCube), c_void_p, c_void_p, c_void_p, c_void_p,
                                           ctypes.c_size_t, c_void_p]
        L.tomo_convnet_loss_grad.argtypes = [POINTER(TomoCube), c_void_p, c_void_p, c_void_p, c_void_p,
                                             POINTER(c_double), c_void_p, ctypes.c_size_t, c_void_p]
        L.tomo_convnet_backward.argtypes = [POINTER(TomoCube), c_void_p, c_void_p, c_void_p, c_void_p,
                                            c_void_p, ctypes.c_size_t, c_void_p]
        L.tomo_adam_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                     c_double, c_double, c_double, c_double, c_void_p]
        L.tomo_set_tuning.argtypes = [POINTER(Tuning)]
        L.tomo_autotune.argtypes = [POINTER(TomoGeometry), c_int32, POINTER(Tuning), c_void_p]
        L.tomo_autotune_data.argtypes = [POINTER(TomoGeometry), c_void_p, c_void_p, c_int32, POINTER(Tuning),
                                         c_void_p]
        L.tomo_get_class_tuning.argtypes = [POINTER(TomoGeometry), POINTER(Tuning), POINTER(c_int32)]
        L.tomo_autotune_clear.argtypes = []
        L.tomo_autotune_clear.restype = None
        L.tomo_batch_create.argtypes = [POINTER(TomoGeometry), c_int32, POINTER(c_void_p)]
        L.tomo_batch_destroy.argtypes = [c_void_p]
        L.tomo_batch_destroy.restype = None
        L.tomo_batch_project.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), c_void_p]
        L.tomo_batch_backproject.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), ctypes.c_int,
                                             c_void_p]
        L.tomo_batch_binning_spills.argtypes = [c_void_p, POINTER(c_int64)]
        L.tomo_batch_items.argtypes = [c_void_p, c_int32]
        L.tomo_batch_items.restype = c_int64
        L.tomo_batch_cg_solve.argtypes = [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(CgParams),
                                          POINTER(CgReport), c_void_p]
        L.tomo_geometry_pixels.argtypes = [POINTER(TomoGeometry)]
        L.tomo_thomson_project.argtypes = [POINTER(TomoGeometry), POINTER(ThomsonParams), c_int32, c_void_p,
                                           c_void_p, c_void_p]
        L.tomo_thomson_backproject.argtypes = [POINTER(TomoGeometry), POINTER(ThomsonParams), c_int32,
                                               c_void_p, c_void_p, c_int32, c_void_p]
        _lib = L
    return _lib


def _check(rc):
    if rc != TOMO_OK:
        raise TomoError(rc, lib().tomo_last_error().decode())


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_f32(t, numel, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda:
        raise ValueError(f"{name} must be a float32 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return c_void_p(t.data_ptr())


class DeviceGeometry:
    """Marshals a geometry description (box, views, masks) into a
    tomo_geometry.  ``geom`` needs the attributes n, lo, hi, views (V x 16:
    obs, w, u, v, cdelt, crpix), npix (V x 2), view_frame (or None), nframes,
    data_mask (or None) and map_mask (or None), and may have obstacle
    ((cx, cy, cz, R) of an opaque sphere, or None) and gains (one per view,
    or None); masks are copied to the device once."""

    def __init__(self, geom, device="cuda"):
        self.n = tuple(int(k) for k in geom.n)
        self.nframes = int(getattr(geom, "nframes", 1) or 1)
        views = np.asarray(geom.views, dtype=np.float64)
        npix = np.asarray(geom.npix, dtype=np.int64)
        vf = getattr(geom, "view_frame", None)
        self.nviews = views.shape[0]
        arr = (TomoView * self.nviews)()
        for k in range(self.nviews):
            row = views[k]
            tv = arr[k]
            for a in range(3):
                tv.obs[a], tv.w[a], tv.u[a], tv.v[a] = row[a], row[3 + a], row[6 + a], row[9 + a]
            tv.cdelt[0], tv.cdelt[1] = row[12], row[13]
            tv.crpix[0], tv.crpix[1] = row[14], row[15]
            tv.ncol, tv.nrow = int(npix[k, 0]), int(npix[k, 1])
            tv.frame = 0 if vf is None else int(vf[k])
        self._views = arr
        self.npix = int(np.sum(npix[:, 0] * npix[:, 1]))
        self.nvox = self.n[0] * self.n[1] * self.n[2]
        self.data_mask = self._mask(getattr(geom, "data_mask", None), self.npix, device)
        self.map_mask = self._mask(getattr(geom, "map_mask", None), self.nvox, device)
        cube = TomoCube(self.n[0], self.n[1], self.n[2], self.nframes,
                        (c_double * 3)(*np.asarray(geom.lo, dtype=np.float64)),
                        (c_double * 3)(*np.asarray(geom.hi, dtype=np.float64)))
        ob = getattr(geom, "obstacle", None)
        self._obstacle = None
        if ob is not None:
            ob = np.asarray(ob, dtype=np.float64).reshape(4)
            self._obstacle = TomoObstacle((c_double * 3)(*ob[:3]), float(ob[3]))
        gn = getattr(geom, "gains", None)
        self._gains = None
        if gn is not None:
            gn = np.asarray(gn, dtype=np.float64).reshape(-1)
            if gn.size != self.nviews:
                raise ValueError(f"{gn.size} gains for {self.nviews} views")
            self._gains = (c_double * self.nviews)(*gn)
        self.g = TomoGeometry(cube, self.nviews, 0, arr,
                              None if self.data_mask is None else self.data_mask.data_ptr(),
                              None if self.map_mask is None else self.map_mask.data_ptr(),
                              None if self._obstacle is None else ctypes.pointer(self._obstacle),
                              None if self._gains is None else self._gains)

    @staticmethod
    def _mask(m, numel, device):
        if m is None:
            return None
        t = torch.as_tensor(np.ascontiguousarray(m).astype(np.uint8).ravel()).to(device)
        if t.numel() != numel:
            raise ValueError(f"mask has {t.numel()} entries, expected {numel}")
        return t

    @property
    def cube_shape(self):
        nx, ny, nz = self.n
        return (self.nframes, nz, ny, nx) if self.nframes > 1 else (nz, ny, nx)

    @property
    def ref(self):
        return ctypes.byref(self.g)

    def validate(self):
        _check(lib().tomo_validate_geometry(self.ref))


def project(geom: DeviceGeometry, cube: torch.Tensor, out: torch.Tensor | None = None):
    """Images = P M cube (one value per pixel, views concatenated)."""
    if out is None:
        out = torch.empty(geom.npix, dtype=torch.float32, device=cube.device)
    c = _dev_f32(cube, geom.nvox * geom.nframes, "cube")
    o = _dev_f32(out, geom.npix, "out")
    _check(lib().tomo_project(geom.ref, c, o, _stream()))
    return out


def backproject(geom: DeviceGeometry, images: torch.Tensor, out: torch.Tensor | None = None,
                accumulate: bool = False, strategy: int = BP_AUTO):
    """Cube = M P^T images (or += with accumulate)."""
    if out is None:
        out = torch.empty(geom.cube_shape, dtype=torch.float32, device=images.device)
    y = _dev_f32(images, geom.npix, "images")
    o = _dev_f32(out, geom.nvox * geom.nframes, "out")
    _check(lib().tomo_backproject_ex(geom.ref, y, o, int(bool(accumulate)), int(strategy), _stream()))
    return out


def backproject_noalloc(geom: DeviceGeometry, images: torch.Tensor, out: torch.Tensor,
                        accumulate: bool = False):
    """Cube = M P^T images (or += with accumulate) through the allocation-free
    entry point: the blocked transpose with the library's static scratch
    array.  `out` must be given (nothing is allocated)."""
    y = _dev_f32(images, geom.npix, "images")
    o = _dev_f32(out, geom.nvox * geom.nframes, "out")
    _check(lib().tomo_backproject_noalloc(geom.ref, y, o, int(bool(accumulate)), _stream()))
    return out


def get_tuning() -> dict:
    t = Tuning()
    _check(lib().tomo_get_tuning(ctypes.byref(t)))
    out = {k: getattr(t, k) for k, _ in Tuning._fields_}
    out["bp_block"] = tuple(t.bp_block)
    return out


def set_tuning(**kw) -> dict:
    """Change launch tuning fields (see tomo_tuning); returns the previous
    settings."""
    old = get_tuning()
    new = dict(old)
    for k, v in kw.items():
        if k not in new:
            raise KeyError(k)
        new[k] = tuple(int(e) for e in v) if k == "bp_block" else int(v)
    t = Tuning(**{k: v for k, v in new.items() if k != "bp_block"})
    for a in range(3):
        t.bp_block[a] = new["bp_block"][a]
    _check(lib().tomo_set_tuning(ctypes.byref(t)))
    return old


def _tuning_dict(t: Tuning) -> dict:
    out = {k: getattr(t, k) for k, _ in Tuning._fields_}
    out["bp_block"] = tuple(t.bp_block)
    return out


def autotune(geom: DeviceGeometry, reps: int = 3, cube: torch.Tensor | None = None,
             images: torch.Tensor | None = None) -> dict:
    """Time the launch candidates on this geometry (on the given cube and
    images, else on a cube of ones and its projection) and keep the fastest
    for its size class if it beats the process-wide tuning
    (tomo_autotune / tomo_autotune_data); returns the chosen tuning."""
    t = Tuning()
    if cube is not None and images is not None:
        _check(lib().tomo_autotune_data(geom.ref, _dev_f32(cube, geom.nvox * geom.nframes, "cube"),
                                        _dev_f32(images, geom.npix, "images"), int(reps), ctypes.byref(t),
                                        _stream()))
    else:
        _check(lib().tomo_autotune(geom.ref, int(reps), ctypes.byref(t), _stream()))
    return _tuning_dict(t)


def class_tuning(geom: DeviceGeometry):
    """(tuning in effect for this geometry, whether the autotuner chose it)."""
    t = Tuning()
    tuned = c_int32(0)
    _check(lib().tomo_get_class_tuning(geom.ref, ctypes.byref(t), ctypes.byref(tuned)))
    return _tuning_dict(t), bool(tuned.value)


def autotune_clear():
    lib().tomo_autotune_clear()


def _ptrs(tensors, numels, name):
    arr = (c_void_p * len(tensors))()
    for k, (t, n) in enumerate(zip(tensors, numels)):
        arr[k] = _dev_f32(t, n, f"{name}[{k}]").value
    return arr


def _height(height):
    """tomo_height from (cx, cy, cz, offset), or None."""
    if height is None:
        return None
    h = np.asarray(height, dtype=np.float64).reshape(4)
    return TomoHeight((c_double * 3)(*h[:3]), float(h[3]))


def _cg_params(lam_r, lam_t, max_iter, rtol, check_every, use_graph, x0_given, height=None, keep=None):
    """CgParams; a height struct is appended to ``keep`` (the caller holds it
    until the call returns)."""
    p = CgParams()
    lib().tomo_cg_default_params(ctypes.byref(p))
    p.lambda_r, p.lambda_t, p.max_iter, p.rtol = lam_r, lam_t, int(max_iter), rtol
    p.check_every, p.use_graph, p.x0_given = int(check_every), int(bool(use_graph)), int(bool(x0_given))
    h = _height(height)
    if h is not None:
        keep.append(h)
        p.height = ctypes.pointer(h)
    return p


_REPORT_KEYS = ("iters", "status", "fell_back", "n_project", "n_backproject", "rel_res", "true_rel_res",
                "bnorm", "ms_project", "ms_backproject")


class Batch:
    """Several independent systems (DeviceGeometry each): one persistent P^T
    launch over all of them, P through each system's own launch
    (tomo_batch_*)."""

    def __init__(self, geoms):
        self.geoms = list(geoms)  # keeps the masks alive
        n = len(self.geoms)
        arr = (TomoGeometry * n)(*[g.g for g in self.geoms])
        self._arr = arr
        self.h = c_void_p()
        _check(lib().tomo_batch_create(arr, n, ctypes.byref(self.h)))

    def close(self):
        if self.h:
            lib().tomo_batch_destroy(self.h)
            self.h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def items(self, which: int) -> int:
        return int(lib().tomo_batch_items(self.h, int(which)))

    def spills(self) -> int:
        c = c_int64(0)
        _check(lib().tomo_batch_binning_spills(self.h, ctypes.byref(c)))
        return int(c.value)

    def project(self, cubes, outs=None):
        if outs is None:
            outs = [torch.empty(g.npix, dtype=torch.float32, device=c.device) for g, c in zip(self.geoms, cubes)]
        src = _ptrs(cubes, [g.nvox * g.nframes for g in self.geoms], "cubes")
        dst = _ptrs(outs, [g.npix for g in self.geoms], "images")
        _check(lib().tomo_batch_project(self.h, src, dst, _stream()))
        return outs

    def backproject(self, images, outs=None, accumulate=False):
        if outs is None:
            outs = [torch.empty(g.cube_shape, dtype=torch.float32, device=y.device)
                    for g, y in zip(self.geoms, images)]
        src = _ptrs(images, [g.npix for g in self.geoms], "images")
        dst = _ptrs(outs, [g.nvox * g.nframes for g in self.geoms], "cubes")
        _check(lib().tomo_batch_backproject(self.h, src, dst, int(bool(accumulate)), _stream()))
        return outs

    def cg_solve(self, ys, x0s=None, *, lam_r=1e-2, lam_t=0.0, max_iter=50, rtol=0.0, check_every=10,
                 use_graph=False, outs=None, heights=None, time_kernels=False):
        """CG on every system at once; lam_r, lam_t, max_iter, rtol may be
        per-system lists, heights a per-system list of (cx, cy, cz, offset)
        or None (height-weighted spatial prior).  With time_kernels, every
        report's ms_project / ms_backproject hold the total time of the
        batched P / P^T launches of the iterations (shared by all systems).
        Returns (xs, reports)."""
        n = len(self.geoms)
        per = lambda v: list(v) if isinstance(v, (list, tuple)) else [v] * n  # noqa: E731
        lr, lt, mi, rt = per(lam_r), per(lam_t), per(max_iter), per(rtol)
        hs = [None] * n if heights is None else list(heights)
        keep = []
        if outs is None:
            outs = [torch.empty(g.cube_shape, dtype=torch.float32, device=y.device) for g, y in zip(self.geoms, ys)]
        if x0s is not None:
            for o, x0 in zip(outs, x0s):
                o.copy_(x0.reshape(o.shape))
        params = (CgParams * n)(*[_cg_params(lr[k], lt[k], mi[k], rt[k], check_every, use_graph, x0s is not None,
                                             hs[k], keep)
                                  for k in range(n)])
        hists = [(c_double * (int(mi[k]) + 1))() for k in range(n)]
        reps = (CgReport * n)()
        for k in range(n):
            reps[k].history = hists[k]
            reps[k].history_cap = int(mi[k]) + 1
            reps[k].time_kernels = int(bool(time_kernels))
        src = _ptrs(ys, [g.npix for g in self.geoms], "y")
        dst = _ptrs(outs, [g.nvox * g.nframes for g in self.geoms], "x")
        _check(lib().tomo_batch_cg_solve(self.h, src, dst, params, reps, _stream()))
        out = []
        for k in range(n):
            d = {key: getattr(reps[k], key) for key in _REPORT_KEYS}
            d["history"] = np.ctypeslib.as_array(hists[k])[:reps[k].history_len].copy()
            out.append(d)
        return outs, out


def binning_spills(geom: DeviceGeometry) -> int:
    """Binned back-projection writes that missed their LDS box (must be 0)."""
    n = c_int64(0)
    _check(lib().tomo_binning_spills(geom.ref, ctypes.byref(n)))
    return int(n.value)


def count_crossings(geom: DeviceGeometry) -> int:
    tot = c_int64(0)
    _check(lib().tomo_count_crossings(geom.ref, ctypes.byref(tot), _stream()))
    return int(tot.value)


def trace_ray(geom: DeviceGeometry, view: int, col: int, row: int):
    """Segments of one pixel's ray from the GPU walk: (flat voxel index,
    length, parametric length)."""
    cap = sum(geom.n) + 3
    idx = (c_int32 * cap)()
    ln = (c_double * cap)()
    dp = (c_double * cap)()
    n = c_int32(0)
    _check(lib().tomo_trace_ray(geom.ref, view, col, row, idx, ln, dp, cap, ctypes.byref(n)))
    k = n.value
    return (np.ctypeslib.as_array(idx)[:k].copy(), np.ctypeslib.as_array(ln)[:k].copy(),
            np.ctypeslib.as_array(dp)[:k].copy())


def _thomson_params(u, scale, sun):
    sun = np.asarray(sun, dtype=np.float64).reshape(4)
    return ThomsonParams(float(u), float(scale), (c_double * 3)(*sun[:3]), float(sun[3]))


def thomson_project(geom: DeviceGeometry, ne: torch.Tensor, u: float = 0.6, kind: str = "pB",
                    scale: float = 1.0, sun=(0.0, 0.0, 0.0, 1.0), out: torch.Tensor | None = None):
    """Thomson-scattering images T n_e (kind "pB": scale O P M n_e; "B":
    scale (P M' - O P M) n_e); sun = (cx, cy, cz, R_sun) in box units."""
    if out is None:
        out = torch.empty(geom.npix, dtype=torch.float32, device=ne.device)
    t = _thomson_params(u, scale, sun)
    _check(lib().tomo_thomson_project(geom.ref, ctypes.byref(t), THOMSON_KINDS[kind],
                                      _dev_f32(ne, geom.nvox * geom.nframes, "ne"),
                                      _dev_f32(out, geom.npix, "out"), _stream()))
    return out


def thomson_backproject(geom: DeviceGeometry, images: torch.Tensor, u: float = 0.6, kind: str = "pB",
                        scale: float = 1.0, sun=(0.0, 0.0, 0.0, 1.0), out: torch.Tensor | None = None,
                        accumulate: bool = False):
    """Transpose T^T y of thomson_project (or += with accumulate)."""
    if out is None:
        out = torch.empty(geom.cube_shape, dtype=torch.float32, device=images.device)
    t = _thomson_params(u, scale, sun)
    _check(lib().tomo_thomson_backproject(geom.ref, ctypes.byref(t), THOMSON_KINDS[kind],
                                          _dev_f32(images, geom.npix, "images"),
                                          _dev_f32(out, geom.nvox * geom.nframes, "out"),
                                          int(bool(accumulate)), _stream()))
    return out


def apply_prior(geom: DeviceGeometry, x: torch.Tensor, lam_r: float, lam_t: float = 0.0,
                out: torch.Tensor | None = None, accumulate: bool = False, height=None):
    """out (+)= lam_r D^T D x + lam_t D_t^T D_t x, or with height = (cx, cy,
    cz, offset) lam_r R D^T D R x + lam_t D_t^T D_t x (R the voxel heights)."""
    if out is None:
        out = torch.empty_like(x)
    n = geom.nvox * geom.nframes
    if height is None:
        _check(lib().tomo_apply_prior(ctypes.byref(geom.g.cube), lam_r, lam_t, _dev_f32(x, n, "x"),
                                      _dev_f32(out, n, "out"), int(bool(accumulate)), _stream()))
    else:
        h = _height(height)
        _check(lib().tomo_apply_height_prior(ctypes.byref(geom.g.cube), ctypes.byref(h), lam_r, lam_t,
                                             _dev_f32(x, n, "x"), _dev_f32(out, n, "out"),
                                             int(bool(accumulate)), _stream()))
    return out


def cg_solve(geom: DeviceGeometry, y: torch.Tensor, x0: torch.Tensor | None = None, *,
             lam_r: float = 1e-2, lam_t: float = 0.0, max_iter: int = 50, rtol: float = 0.0,
             check_every: int = 10, use_graph: bool = False, precond: torch.Tensor | None = None,
             fallback_window: int = 3, min_drop: float = 1e-6, bp_strategy: int = BP_AUTO,
             time_kernels: bool = False, out: torch.Tensor | None = None,
             record_x: torch.Tensor | None = None, record_r: torch.Tensor | None = None, height=None,
             workspace: torch.Tensor | None = None):
    """Solve M (P^T G^2 P + lam_r R D^T D R + lam_t D_t^T D_t) M x = M P^T G y
    (G the geometry's gains; R the voxel heights for height = (cx, cy, cz,
    offset), else the identity).  workspace: a CUDA uint8 tensor of at least
    cg_workspace_bytes(...) bytes for all of the solve's device buffers, or
    None (stream-ordered scratch).  Returns (x, report dict)."""
    p = CgParams()
    lib().tomo_cg_default_params(ctypes.byref(p))
    h = _height(height)
    if h is not None:
        p.height = ctypes.pointer(h)
    p.lambda_r, p.lambda_t, p.max_iter, p.rtol = lam_r, lam_t, int(max_iter), rtol
    p.check_every, p.use_graph = int(check_every), int(bool(use_graph))
    p.fallback_window, p.min_drop, p.bp_strategy = int(fallback_window), min_drop, int(bp_strategy)
    if precond is not None:
        p.precond = _dev_f32(precond, precond.numel(), "precond")
    if record_x is not None or record_r is not None:
        count = (record_x if record_x is not None else record_r).shape[0]
        nv = geom.nvox * geom.nframes
        p.record_count = int(count)
        if record_x is not None:
            p.record_x = _dev_f32(record_x, count * nv, "record_x")
        if record_r is not None:
            p.record_r = _dev_f32(record_r, count * nv, "record_r")
    if workspace is not None:
        if not workspace.is_cuda or not workspace.is_contiguous():
            raise ValueError("workspace must be a contiguous CUDA tensor")
        p.workspace = workspace.data_ptr()
        p.workspace_bytes = workspace.numel() * workspace.element_size()
    if out is None:
        out = torch.empty(geom.cube_shape, dtype=torch.float32, device=y.device)
    if x0 is not None:
        out.copy_(x0.reshape(out.shape))
        p.x0_given = 1
    hist = (c_double * (int(max_iter) + 1))()
    rep = CgReport()
    rep.history = hist
    rep.history_cap = int(max_iter) + 1
    rep.time_kernels = int(bool(time_kernels))
    _check(lib().tomo_cg_solve(geom.ref, _dev_f32(y, geom.npix, "y"),
                               _dev_f32(out, geom.nvox * geom.nframes, "x"), ctypes.byref(p),
                               ctypes.byref(rep), _stream()))
    report = {k: getattr(rep, k) for k in _REPORT_KEYS}
    report["history"] = np.ctypeslib.as_array(hist)[:rep.history_len].copy()
    return out, report


def cg_workspace_bytes(geom: DeviceGeometry, *, max_iter: int = 50, precond: torch.Tensor | None = None,
                       bp_strategy: int = BP_AUTO) -> int:
    """Device workspace bytes cg_solve takes with these settings
    (tomo_cg_workspace_bytes); 0 for settings it rejects."""
    p = CgParams()
    lib().tomo_cg_default_params(ctypes.byref(p))
    p.max_iter, p.bp_strategy = int(max_iter), int(bp_strategy)
    if precond is not None:
        p.precond = _dev_f32(precond, precond.numel(), "precond")
    return int(lib().tomo_cg_workspace_bytes(geom.ref, ctypes.byref(p)))


class ConvNet:
    """Device-side runner for the preconditioner network on one volume shape
    (nx, ny, nz): owns the workspace; parameters are a float32 CUDA tensor of
    NPARAMS values (w1, b1, w2, b2, w3, b3 as in include/tomo.h)."""

    def __init__(self, shape_zyx, device="cuda"):
        nz, ny, nx = (int(k) for k in shape_zyx)
        self.cube = TomoCube(nx, ny, nz, 1, (c_double * 3)(0, 0, 0), (c_double * 3)(1, 1, 1))
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        nbytes = lib().tomo_convnet_workspace_bytes(ctypes.byref(self.cube))
        if nbytes == 0:
            raise ValueError("invalid volume shape")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)

    def forward(self, params, x, out=None):
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=x.device)
        _check(lib().tomo_convnet_forward(ctypes.byref(self.cube), _dev_f32(params, NPARAMS, "params"),
                                          _dev_f32(x, self.n, "x"), _dev_f32(out, self.n, "out"),
                                          c_void_p(self.ws.data_ptr()), self.ws.numel(), _stream()))
        return out

    def loss_grad(self, params, x, target, grad=None, want_loss=True):
        """grad of mean((N(x) - target)^2) w.r.t. params; returns (loss or None, grad)."""
        if grad is None:
            grad = torch.empty(NPARAMS, dtype=torch.float32, device=x.device)
        loss = c_double(0.0)
        _check(lib().tomo_convnet_loss_grad(ctypes.byref(self.cube), _dev_f32(params, NPARAMS, "params"),
                                            _dev_f32(x, self.n, "x"), _dev_f32(target, self.n, "target"),
                                            _dev_f32(grad, NPARAMS, "grad"),
                                            ctypes.byref(loss) if want_loss else None,
                                            c_void_p(self.ws.data_ptr()), self.ws.numel(), _stream()))
        return (loss.value if want_loss else None), grad

    def backward(self, params, x, dout, grad=None):
        """grad of sum(dout * N(x)) w.r.t. params (dout: d loss / d N(x))."""
        if grad is None:
            grad = torch.empty(NPARAMS, dtype=torch.float32, device=x.device)
        _check(lib().tomo_convnet_backward(ctypes.byref(self.cube), _dev_f32(params, NPARAMS, "params"),
                                           _dev_f32(x, self.n, "x"), _dev_f32(dout, self.n, "dout"),
                                           _dev_f32(grad, NPARAMS, "grad"), c_void_p(self.ws.data_ptr()),
                                           self.ws.numel(), _stream()))
        return grad


def adam_step(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    n = params.numel()
    _check(lib().tomo_adam_step(_dev_f32(params, n, "params"), _dev_f32(grad, n, "grad"),
                                _dev_f32(m, n, "m"), _dev_f32(v, n, "v"), n, int(step), lr, beta1,
                                beta2, eps, _stream()))


def view_from_wcs(dsun, hgln_deg, hglt_deg, crval1_as, crval2_as, crota_deg, cdelt1_as,
                  cdelt2_as, crpix1, crpix2, ncol, nrow):
    """View row (16 numbers) and (ncol, nrow) from helioprojective TAN WCS keywords."""
    tv = TomoView()
    _check(lib().tomo_view_from_wcs(dsun, hgln_deg, hglt_deg, crval1_as, crval2_as, crota_deg,
                                    cdelt1_as, cdelt2_as, crpix1, crpix2, ncol, nrow,
                                    ctypes.byref(tv)))
    row = np.array(list(tv.obs) + list(tv.w) + list(tv.u) + list(tv.v) + list(tv.cdelt)
                   + list(tv.crpix))
    return row, np.array([tv.ncol, tv.nrow], dtype=np.int32)


def validate(geom: DeviceGeometry) -> int:
    """Status code of the library's geometry check (no GPU work)."""
    return int(lib().tomo_validate_geometry(geom.ref))


def status_string(status: int) -> str:
    return lib().tomo_status_string(int(status)).decode()
