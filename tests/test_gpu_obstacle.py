"""GPU parity of the obstacle variant (lines of sight end where they enter
an opaque sphere, the photosphere: the projector's obstacle variant in
Sec. "Fast Parallelized Projector", integration stopped at the photosphere
in Sec. "Performance") against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import (CODES, STRATEGIES, assert_p_close, flat_index, length_resolution, need_gpu,
                         oracle_pixels, parity_full, sample_pixels, to_dev, to_host)

pytestmark = pytest.mark.gpu

SUN = np.array([0.0, 0.0, 0.0, 1.0])


@pytest.fixture(scope="module")
def tomo():
    return need_gpu()


def _near(obstacle=SUN):
    """16^3 cube on [-1.5, 1.5]^3 seen from 4 R_sun by 6 views of 24 x 20
    pixels over 3.2 R_sun: the sphere hides part of the box and many lines
    of sight pass beside it."""
    n, lo, hi = ts.box(16, 1.5)
    views, npix = ts.make_views([0.0, 50.0, 110.0, 190.0, 250.0, 320.0], (24, 20), 3.2, lat=15.0, dist=4.0)
    return ts.Geometry(n, lo, hi, views, npix, obstacle=None if obstacle is None else np.array(obstacle))


def test_near_views_every_pixel_and_voxel(tomo, ora):
    g = _near()
    rng = np.random.default_rng(40)
    parity_full(tomo, ora, g, rng.uniform(size=g.cube_shape()), rng.normal(size=g.nrays))


def test_offset_sphere_and_masks(tomo, ora):
    """A sphere off the box centre, a data mask and a map mask together."""
    g0 = _near(obstacle=np.array([0.3, -0.2, 0.1, 0.8]))
    rng = np.random.default_rng(41)
    dm = (rng.uniform(size=g0.nrays) > 0.25).astype(np.uint8)
    mm = (rng.uniform(size=g0.cube_shape()) > 0.2).astype(np.uint8)
    g = ts.Geometry(g0.n, g0.lo, g0.hi, g0.views, g0.npix, data_mask=dm, map_mask=mm, obstacle=g0.obstacle)
    parity_full(tomo, ora, g, rng.uniform(size=g.cube_shape()), rng.normal(size=g.nrays))


def test_crossing_counts_and_the_cut(tomo, ora):
    g = _near()
    free = ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix)
    n_ob = tomo.count_crossings(tomo.DeviceGeometry(g))
    assert n_ob == ora.count_crossings(g)
    assert n_ob < tomo.count_crossings(tomo.DeviceGeometry(free))


def test_observer_inside_sees_nothing(tomo, ora):
    g0 = _near()
    g = ts.Geometry(g0.n, g0.lo, g0.hi, g0.views, g0.npix, obstacle=np.array([0.0, 0.0, 0.0, 5.0]))
    dg = tomo.DeviceGeometry(g)
    assert tomo.count_crossings(dg) == 0
    img = to_host(tomo.project(dg, to_dev(np.ones(g.cube_shape()))))
    assert np.all(img == 0.0)
    y = to_dev(np.random.default_rng(42).normal(size=g.nrays))
    for strat in STRATEGIES:
        assert np.all(to_host(tomo.backproject(dg, y, strategy=CODES[strat])) == 0.0), strat


def test_euvi_two_views_with_the_photosphere(tomo, ora):
    """EUVI-like 128^3 with the unit sphere masked, two views of 512^2 from
    215 R_sun, and the photosphere as obstacle: the disc's lines of sight
    stop at its near side.  Every pixel and voxel compared."""
    wl = ts.euvi()
    g0 = wl.geom.subset([0, 13])
    g = ts.Geometry(g0.n, g0.lo, g0.hi, g0.views, g0.npix, map_mask=g0.map_mask, obstacle=SUN.copy())
    y = np.random.default_rng(43).normal(size=g.nrays)
    parity_full(tomo, ora, g, wl.x, y)


def test_euvi_full_size_sampled(tomo, ora):
    """All 28 views of 512^2 with the photosphere: P on 3000 sampled pixels."""
    wl = ts.euvi()
    g0 = wl.geom
    g = ts.Geometry(g0.n, g0.lo, g0.hi, g0.views, g0.npix, map_mask=g0.map_mask, obstacle=SUN.copy())
    dg = tomo.DeviceGeometry(g)
    img = to_host(tomo.project(dg, to_dev(wl.x)))
    pix = sample_pixels(g, 3000, 44)
    got = np.array([img[flat_index(g, *p)] for p in pix])
    # the oracle's per-pixel walk, cut at the sphere
    vals, absv = [], []
    xf = wl.x.reshape(-1) * g.map_mask.reshape(-1)
    for v, col, row in pix:
        d = ora.pixel_direction(g.views[v], g.npix[v], col, row)
        idx, ln, _ = ora.trace_ray(g.n, g.lo, g.hi, g.views[v][0:3], d, SUN)
        vals.append(float(np.sum(ln * xf[idx])))
        absv.append(float(np.sum(ln * np.abs(xf[idx]))))
    assert_p_close(got, np.array(vals), np.array(absv), atol=length_resolution(g) * np.abs(wl.x).max())


def test_batch_with_an_obstacle(tomo, ora):
    """Batched P and P^T of a system with the obstacle next to one without
    equal the per-system calls bit for bit."""
    ga, gb = _near(), _near(obstacle=None)
    dga, dgb = tomo.DeviceGeometry(ga), tomo.DeviceGeometry(gb)
    rng = np.random.default_rng(45)
    xa, xb = to_dev(rng.uniform(size=ga.cube_shape())), to_dev(rng.uniform(size=gb.cube_shape()))
    ya, yb = to_dev(rng.normal(size=ga.nrays)), to_dev(rng.normal(size=gb.nrays))
    batch = tomo.Batch([dga, dgb])
    try:
        pa, pb = batch.project([xa, xb])
        ba, bb = batch.backproject([ya, yb])
        np.testing.assert_array_equal(to_host(pa), to_host(tomo.project(dga, xa)))
        np.testing.assert_array_equal(to_host(pb), to_host(tomo.project(dgb, xb)))
        np.testing.assert_array_equal(to_host(ba), to_host(tomo.backproject(dga, ya, strategy=CODES["blocked"])))
        np.testing.assert_array_equal(to_host(bb), to_host(tomo.backproject(dgb, yb, strategy=CODES["blocked"])))
    finally:
        batch.close()


def test_adjoint_identity(tomo):
    g = _near()
    dg = tomo.DeviceGeometry(g)
    rng = np.random.default_rng(46)
    x, y = rng.normal(size=g.cube_shape()), rng.normal(size=g.nrays)
    px = to_host(tomo.project(dg, to_dev(x)))
    pty = to_host(tomo.backproject(dg, to_dev(y), strategy=CODES["blocked"]))
    lhs, rhs = float(np.dot(px, y)), float(np.sum(x * pty))
    assert abs(lhs - rhs) <= 1e-5 * (float(np.dot(np.abs(px), np.abs(y))) + 1e-30)
