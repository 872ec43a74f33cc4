"""GPU parity of the widened features used together, against the FP64
oracle through the C ABI: the Thomson operators of a geometry with the
photosphere as obstacle and per-instrument gains, P and every P^T strategy
with an obstacle, gains and both masks, and the graph-captured batched CG
of a time-dependent system with the height-weighted prior next to a
two-instrument system."""
import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import assert_p_close, length_resolution, need_gpu, parity_full, to_dev, to_host

pytestmark = pytest.mark.gpu

SUN = np.array([0.0, 0.0, 0.0, 1.0])


@pytest.fixture(scope="module")
def tomo():
    return need_gpu()


def _coronagraph():
    """32^3 on [-4, 4]^3 R_sun, the unit sphere masked and opaque; two
    instruments (3 views of 48^2 at gain 1, 2 views of 40^2 at gain 0.55),
    the detector annulus 1.4-4 R_sun kept."""
    nn, lo, hi = ts.box(32, 4.0)
    va, pa = ts.make_views([0.0, 120.0, 240.0], (48, 48), 8.0, lat=7.0)
    vb, pb = ts.make_views([60.0, 180.0], (40, 40), 8.0, lat=-5.0)
    views, npix = np.concatenate([va, vb]), np.concatenate([pa, pb])
    return ts.Geometry(nn, lo, hi, views, npix, data_mask=ts.annulus_data_mask(views, npix, 1.4, 4.0),
                       map_mask=ts.sphere_map_mask(nn, lo, hi, 1.0), obstacle=SUN.copy(),
                       gains=np.array([1.0, 1.0, 1.0, 0.55, 0.55]))


@pytest.mark.parametrize("kind", ["pB", "B"])
def test_thomson_with_obstacle_and_gains(tomo, ora, kind):
    g = _coronagraph()
    u, scale = 0.63, 3.0
    rng = np.random.default_rng(70)
    x, y = rng.uniform(size=g.cube_shape()), rng.normal(size=g.nrays)
    m, mp = ora.thomson_voxel_weights(g, u)
    o = ora.thomson_pixel_weights(g)
    ax, ay = np.abs(x), np.abs(y)
    if kind == "pB":
        fa = scale * o * ora.project(g, ax * m)
        ba = scale * m * ora.backproject(g, o * ay)
    else:
        fa = scale * (ora.project(g, ax * mp) + o * ora.project(g, ax * m))
        ba = scale * (mp * ora.backproject(g, ay) + m * ora.backproject(g, o * ay))
    dg = tomo.DeviceGeometry(g)
    res = length_resolution(g)
    got = to_host(tomo.thomson_project(dg, to_dev(x), u, kind, scale))
    assert_p_close(got, ora.thomson_project(g, x, u, kind, scale), fa, what=f"T_{kind}",
                   atol=res * float(np.max(np.abs(fa))))
    assert np.count_nonzero(got) > 0.2 * g.nrays
    gotb = to_host(tomo.thomson_backproject(dg, to_dev(y), u, kind, scale))
    assert_p_close(gotb, ora.thomson_backproject(g, y, u, kind, scale), ba, rtol=1e-4, what=f"T_{kind}^T",
                   atol=res * float(np.max(np.abs(ba))))


def test_obstacle_gains_masks_every_strategy(tomo, ora):
    g = _coronagraph()
    rng = np.random.default_rng(71)
    parity_full(tomo, ora, g, rng.uniform(size=g.cube_shape()), rng.normal(size=g.nrays))


def test_batched_graph_cg_frames_height_and_gains(tomo, ora):
    """Graph-captured batched CG of two systems: three time frames coupled
    by the temporal prior under the height-weighted spatial prior (offset -1:
    altitude above the photosphere), and a two-instrument static system with
    the plain prior; 12 iterations each against the oracle's CG."""
    wl = ts.tiny()
    g0 = wl.geom
    vf = (np.arange(g0.nviews) % 3).astype(np.int32)
    mm = ts.sphere_map_mask(g0.n, g0.lo, g0.hi, 0.6)
    ga = ts.Geometry(g0.n, g0.lo, g0.hi, g0.views, g0.npix, vf, 3, None, mm)
    xa = np.stack([wl.x * (1 + 0.1 * f) for f in range(3)])
    ya = ora.project(ga, xa).astype(np.float32).astype(np.float64)
    gb = g0.subset(np.arange(g0.nviews))
    gb.gains = np.where(np.arange(gb.nviews) < 4, 0.8, 1.3)
    yb = ora.project(gb, wl.x).astype(np.float32).astype(np.float64)
    ha = (0.0, 0.0, 0.0, -1.0)
    dga, dgb = tomo.DeviceGeometry(ga), tomo.DeviceGeometry(gb)
    batch = tomo.Batch([dga, dgb])
    try:
        xs, reps = batch.cg_solve([to_dev(ya), to_dev(yb)], lam_r=[1e-2, 1e-2], lam_t=[10.0, 0.0], max_iter=12,
                                  use_graph=True, check_every=4, heights=[ha, None])
    finally:
        batch.close()
    for xg, rep, g, y, lt, h in zip(xs, reps, (ga, gb), (ya, yb), (10.0, 0.0), (ha, None)):
        xo, ho = ora.cg(ora.normal_operator(g, 1e-2, lt, height=h), ora.rhs(g, y), n_iter=12)
        np.testing.assert_allclose(rep["history"], ho, rtol=2e-4)
        assert np.linalg.norm(to_host(xg) - xo) <= 1e-4 * np.linalg.norm(xo)
