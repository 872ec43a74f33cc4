"""Helpers shared by the GPU parity tests (not collected as tests)."""
import dataclasses

import numpy as np
import pytest
import torch

P_RTOL = 1e-5   # per pixel, relative to the oracle's P|x| (stated bound for P)
PT_RTOL = 1e-4  # per voxel, relative to the oracle's P^T|y| (stated bound for P^T)


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_1103_5904_amd as tomo

    return tomo


def to_dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def length_resolution(g):
    """Absolute resolution of the oracle's FP64 segment lengths: each crossing
    parameter t (up to |obs| + box diagonal, with |d| ~ 1) is rounded to
    ~eps * t, so a length carries up to ~2 eps t; with a factor 2 of margin."""
    tmax = np.max(np.linalg.norm(g.views[:, 0:3], axis=1)) + np.linalg.norm(g.hi - g.lo)
    return 4.0 * np.finfo(np.float64).eps * tmax


def assert_p_close(gpu, ora_val, ora_abs, rtol=P_RTOL, what="P", atol=0.0):
    """|gpu - oracle| <= rtol * (P|x|)_ray + atol per entry; entries whose
    P|x| is 0 must be exactly 0 on the GPU.  atol is the oracle's own
    resolution (length_resolution x max |value|), which only matters for
    entries built from segments too short for FP64 to resolve."""
    gpu = np.asarray(gpu, dtype=np.float64).ravel()
    ora_val = np.asarray(ora_val).ravel()
    ora_abs = np.asarray(ora_abs).ravel()
    err = np.abs(gpu - ora_val)
    bound = rtol * ora_abs + atol
    zero = ora_abs == 0
    stray = np.abs(gpu[zero]) > atol  # a sub-resolution near-tie may show on one side only
    assert not np.any(stray), f"{what}: {np.count_nonzero(stray)} untouched entries non-zero"
    bad = err > bound
    if np.any(bad):
        k = np.argmax(err / np.maximum(bound, 1e-300))
        raise AssertionError(f"{what}: {np.count_nonzero(bad)} of {err.size} entries exceed the bound; "
                             f"worst at {k}: gpu {gpu[k]!r} oracle {ora_val[k]!r} bound {bound[k]:.3e}")
    return float(np.max(err / np.where(zero, 1.0, ora_abs)))


def oracle_pixels(ora, g, cube, pix_list):
    """Oracle line integrals for selected pixels only: (values, abs values)
    from the Siddon segments of each pixel's ray."""
    x = np.asarray(cube, dtype=np.float64)
    nvox = g.nvox
    flat = x.reshape(-1)
    vals, absv = [], []
    for v, col, row in pix_list:
        if g.data_mask is not None:
            off = g.view_offsets()[v] + row * g.npix[v][0] + col
            if not g.data_mask[off]:
                vals.append(0.0)
                absv.append(0.0)
                continue
        d = ora.pixel_direction(g.views[v], g.npix[v], col, row)
        idx, ln, _ = ora.trace_ray(g.n, g.lo, g.hi, g.views[v][0:3], d)
        base = 0 if g.view_frame is None else int(g.view_frame[v]) * nvox
        xv = flat[base + idx]
        if g.map_mask is not None:
            xv = xv * g.map_mask.reshape(-1)[idx]
        vals.append(float(np.sum(ln * xv)))
        absv.append(float(np.sum(ln * np.abs(xv))))
    return np.array(vals), np.array(absv)


def sample_pixels(g, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        v = int(rng.integers(0, g.nviews))
        ncol, nrow = (int(t) for t in g.npix[v])
        out.append((v, int(rng.integers(0, ncol)), int(rng.integers(0, nrow))))
    return out


def flat_index(g, v, col, row):
    return int(g.view_offsets()[v] + row * g.npix[v][0] + col)


STRATEGIES = ["blocked", "binned", "atomic"]
CODES = {"blocked": 3, "binned": 2, "atomic": 1}


def parity_full(tomo, ora, g, x, y, strategies=STRATEGIES):
    """Every pixel of P and every voxel of P^T (each back-projection
    strategy) against the oracle.  With gains the bounds scale with |gain|
    (the operators on |x| and |y| taken with |gains|)."""
    dg = tomo.DeviceGeometry(g)
    gains = getattr(g, "gains", None)
    gmax = 1.0 if gains is None else float(np.abs(gains).max())
    ga = g if gains is None else dataclasses.replace(g, gains=np.abs(np.asarray(gains, dtype=np.float64)))
    res = length_resolution(g) * gmax
    img = to_host(tomo.project(dg, to_dev(x)))
    xm = x if g.map_mask is None else x * (g.map_mask if g.nframes == 1 else g.map_mask[None])
    assert_p_close(img, ora.project(g, x), ora.project(ga, np.abs(xm)), atol=res * np.abs(x).max())
    ref, refa = ora.backproject(g, y), ora.backproject(ga, np.abs(y))
    for strat in strategies:
        code = CODES[strat]
        bp = to_host(tomo.backproject(dg, to_dev(y), strategy=code))
        assert_p_close(bp, ref, refa, rtol=1e-4, what=f"P^T ({strat})", atol=res * np.abs(y).max())
        assert tomo.binning_spills(dg) == 0
