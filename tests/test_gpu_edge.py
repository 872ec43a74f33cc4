"""Degenerate and extreme inputs of P, P^T and the solver on the GPU,
against the FP64 oracle: a one-voxel cube, one-voxel-thick slabs, views that
miss the box, a frame no view sees, zero inputs, a view of the largest
detector width the ABI accepts, and rays through a voxel edge line."""
import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import (STRATEGIES, CODES, assert_p_close, length_resolution, need_gpu, parity_full, to_dev,
                         to_host)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tomo():
    return need_gpu()


def _views(specs):
    rows, pix = [], []
    for obs, target, npix, fov in specs:
        r, p = ts.pinhole_view(np.asarray(obs, dtype=np.float64), target=target, npix=npix, fov=fov)
        rows.append(r)
        pix.append(p)
    return np.array(rows), np.array(pix, dtype=np.int32)


def test_one_voxel_cube(tomo, ora):
    """N = 1 along every axis: each ray that hits the box has one segment, its
    chord through the box."""
    views, pix = _views([(ts.observer(lon, lat, 30.0), (0.0, 0.0, 0.0), (9, 7), 2.5)
                         for lon, lat in [(0.0, 0.0), (37.0, 20.0), (200.0, -65.0)]])
    g = ts.Geometry((1, 1, 1), np.full(3, -0.5), np.full(3, 0.5), views, pix)
    x = np.array([[[1.75]]])
    parity_full(tomo, ora, g, x, np.random.default_rng(20).normal(size=g.nrays))


@pytest.mark.parametrize("n", [(1, 40, 3), (33, 1, 17), (5, 6, 1)])
def test_one_voxel_thick_slabs(tomo, ora, n):
    views, pix = _views([(ts.observer(lon, lat, 25.0), (0.1, -0.2, 0.05), (21, 18), 3.0)
                         for lon, lat in [(10.0, 5.0), (95.0, -30.0), (181.0, 60.0), (270.0, 0.0)]])
    g = ts.Geometry(n, np.array([-1.0, -0.8, -0.6]), np.array([0.9, 1.1, 0.7]), views, pix)
    rng = np.random.default_rng(21)
    parity_full(tomo, ora, g, rng.uniform(size=g.cube_shape()), rng.normal(size=g.nrays))


def test_views_that_miss_the_box(tomo, ora):
    """Observers looking away from the box: every P pixel, every P^T voxel and
    the crossing count are exactly zero, with every strategy."""
    views, pix = _views([(ts.observer(0.0, 0.0, 10.0), (20.0, 0.0, 0.0), (16, 16), 1.0),
                         (ts.observer(90.0, 30.0, 10.0), (0.0, 40.0, 25.0), (7, 33), 1.0)])
    g = ts.Geometry((12, 10, 8), np.full(3, -1.0), np.full(3, 1.0), views, pix)
    assert ora.count_crossings(g) == 0
    dg = tomo.DeviceGeometry(g)
    assert tomo.count_crossings(dg) == 0
    rng = np.random.default_rng(22)
    img = to_host(tomo.project(dg, to_dev(rng.uniform(size=g.cube_shape()))))
    assert np.all(img == 0.0)
    y = to_dev(rng.normal(size=g.nrays))
    for strat in STRATEGIES:
        bp = to_host(tomo.backproject(dg, y, strategy=CODES[strat]))
        assert np.all(bp == 0.0), strat


def test_some_rays_miss(tomo, ora):
    """A wide view whose outer pixels pass beside the box, next to a view
    that sees all of it."""
    views, pix = _views([(ts.observer(30.0, 10.0, 8.0), (0.0, 0.0, 0.0), (40, 40), 6.0),
                         (ts.observer(150.0, -10.0, 8.0), (0.0, 0.0, 0.0), (16, 16), 1.5)])
    g = ts.Geometry((10, 11, 12), np.full(3, -1.0), np.full(3, 1.0), views, pix)
    rng = np.random.default_rng(23)
    parity_full(tomo, ora, g, rng.uniform(size=g.cube_shape()), rng.normal(size=g.nrays))


def test_zero_inputs(tomo, ora):
    """P of a zero cube and P^T of a zero image are exactly zero (the
    fixed-point back-projection's scale comes from max |y|, here 0), and CG
    with y = 0 stops at once with x = 0."""
    wl = ts.tiny()
    g = wl.geom
    dg = tomo.DeviceGeometry(g)
    img = to_host(tomo.project(dg, to_dev(np.zeros(g.cube_shape()))))
    assert np.all(img == 0.0)
    for strat in STRATEGIES:
        bp = to_host(tomo.backproject(dg, to_dev(np.zeros(g.nrays)), strategy=CODES[strat]))
        assert np.all(bp == 0.0), strat
    x, rep = tomo.cg_solve(dg, to_dev(np.zeros(g.nrays)), lam_r=1e-2, max_iter=10)
    assert rep["status"] == 0
    assert rep["iters"] == 0
    assert np.all(to_host(x) == 0.0)


def test_one_nonzero_pixel(tomo, ora):
    """P^T of an image with a single non-zero pixel is that ray's segment
    lengths times its value (the fixed-point scale set by one pixel)."""
    wl = ts.tiny()
    g = wl.geom
    dg = tomo.DeviceGeometry(g)
    y = np.zeros(g.nrays)
    k = 3 * 32 * 32 + 15 * 32 + 17
    y[k] = -2.5e-3
    ref, refa = ora.backproject(g, y), ora.backproject(g, np.abs(y))
    assert np.count_nonzero(ref) > 0
    for strat in STRATEGIES:
        bp = to_host(tomo.backproject(dg, to_dev(y), strategy=CODES[strat]))
        assert_p_close(bp, ref, refa, rtol=1e-4, what=f"P^T ({strat})",
                       atol=length_resolution(g) * 2.5e-3)


def test_frame_without_views(tomo, ora):
    """Three frames, the middle one seen by no view: its P^T block is exactly
    zero and the other frames match the oracle."""
    wl = ts.tiny()
    g = wl.geom
    vf = np.where(np.arange(g.nviews) % 2 == 0, 0, 2).astype(np.int32)
    gf = ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, vf, 3)
    rng = np.random.default_rng(24)
    x = np.stack([wl.x * (f + 1) for f in range(3)])
    parity_full(tomo, ora, gf, x, rng.normal(size=g.nrays))
    dg = tomo.DeviceGeometry(gf)
    for strat in STRATEGIES:
        bp = to_host(tomo.backproject(dg, to_dev(rng.normal(size=g.nrays)), strategy=CODES[strat]))
        assert np.all(bp[1] == 0.0), strat


def test_widest_detector(tomo, ora):
    """A 65535 x 2 view (the largest column count) plus a 1 x 700 view: the
    pixel tiling's ragged edges at the extremes, every pixel and voxel checked
    (aim points off the grid lines, so no ray meets a voxel edge exactly)."""
    views, pix = _views([(ts.observer(20.0, 5.0, 12.0), (0.013, -0.021, 0.007), (65535, 2), 2.6),
                         (ts.observer(110.0, -40.0, 12.0), (0.031, 0.017, -0.011), (1, 700), 2.6)])
    g = ts.Geometry((24, 20, 16), np.full(3, -1.0), np.full(3, 1.0), views, pix)
    rng = np.random.default_rng(25)
    parity_full(tomo, ora, g, rng.uniform(size=g.cube_shape()), rng.normal(size=g.nrays))


def test_rays_through_a_voxel_edge_line(tomo, ora):
    """A one-column view aimed at the box centre: all its rays lie in one
    vertical plane that holds the grid's corner line x = y = 0, so every ray
    meets four voxels at once there.  Each side resolves that tie in its own
    FP64 rounding, and a tie resolved the other way leaves a segment of at
    most the length resolution in a neighbour voxel; those add up over the
    column's rays, so the absolute slack is the resolution times sum |y| over
    the view.  The total, sum over voxels of P^T y = sum over rays of y times
    the chord, does not depend on ties; it is held to 1e-6 of sum P^T |y|
    (FP32 output)."""
    views, pix = _views([(ts.observer(110.0, -40.0, 12.0), (0.0, 0.0, 0.0), (1, 700), 2.6)])
    g = ts.Geometry((24, 20, 16), np.full(3, -1.0), np.full(3, 1.0), views, pix)
    y = np.random.default_rng(26).normal(size=g.nrays)
    dg = tomo.DeviceGeometry(g)
    ref, refa = ora.backproject(g, y), ora.backproject(g, np.abs(y))
    atol = length_resolution(g) * np.sum(np.abs(y))
    x = np.random.default_rng(27).uniform(size=g.cube_shape())
    img = to_host(tomo.project(dg, to_dev(x)))
    assert_p_close(img, ora.project(g, x), ora.project(g, x), atol=length_resolution(g))
    for strat in STRATEGIES:
        bp = to_host(tomo.backproject(dg, to_dev(y), strategy=CODES[strat]))
        assert_p_close(bp, ref, refa, rtol=1e-4, what=f"P^T ({strat})", atol=atol)
        tot = float(np.sum(ref))
        assert abs(float(np.sum(bp)) - tot) <= 1e-6 * float(np.sum(refa)), strat
