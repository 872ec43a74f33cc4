"""GPU parity of the height-weighted prior R D^T D R (Eq. srt_inversion) and
of the multi-instrument operator with per-instrument gains (Eq.
two_spacecraft, Eq. lin2space, Eq. srt_multiple_inv) against the FP64
oracle, through the C ABI: the prior stencil, P and every P^T strategy with
gains, the batched launches, the Thomson operators, and CG on the normal
equations with both."""
import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import (CODES, assert_p_close, flat_index, length_resolution, need_gpu, oracle_pixels,
                         parity_full, sample_pixels, to_dev, to_host)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tomo():
    return need_gpu()


def _degree(shape):
    """In-cube 6-neighbour count of every voxel of an (nz, ny, nx) grid."""
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((i > 0).astype(float) + (i < nx - 1) + (j > 0) + (j < ny - 1) + (k > 0) + (k < nz - 1))


def _prior_case(tomo, ora, n, lo, hi, nframes, height, lam_r, lam_t, seed):
    views, npix = ts.make_views([0.0], (1, 1), 1.0)
    vf = np.zeros(1, np.int32) if nframes > 1 else None
    g = ts.Geometry(n, np.array(lo, float), np.array(hi, float), views, npix, vf, nframes)
    dg = tomo.DeviceGeometry(g)
    x = np.random.default_rng(seed).normal(size=dg.cube_shape)
    xf = x.astype(np.float32).astype(np.float64)
    got = to_host(tomo.apply_prior(dg, to_dev(xf), lam_r, lam_t, height=height))
    h = ora.voxel_heights(g, height)
    ref = lam_r * ora.height_prior(xf, h)
    if nframes > 1:
        ref = ref + lam_t * ora.laplacian_t(xf)
    # per voxel: lam_r |h_v| (deg |h_v x_v| + sum |h_n x_n|) + lam_t 4 |x|max,
    # bounded by deg-weighted maxima; FP32 heights and products: ~1e-6 of it
    deg = _degree(g.cube_shape() if nframes == 1 else g.cube_shape()[1:])
    hx = np.abs(h * xf).max()
    scale = lam_r * np.abs(h) * 2.0 * deg * hx + lam_t * 4.0 * np.abs(xf).max()
    err = np.abs(got - ref)
    assert np.all(err <= 2e-6 * scale + 1e-30), float(np.max(err / scale))
    return g, dg, xf, got


def test_height_prior_parity_ragged(tomo, ora):
    """A ragged 13 x 9 x 6 grid in an off-centre box, height centre inside
    the box and offset -1 (heights of both signs)."""
    _prior_case(tomo, ora, (13, 9, 6), [-1.7, -0.4, -1.1], [2.1, 1.3, 0.9], 1, (0.3, -0.2, 0.1, -1.0),
                0.37, 0.0, 20)


def test_height_prior_parity_frames(tomo, ora):
    """Three frames: every frame weighted by the same R, plus the unweighted
    temporal term."""
    _prior_case(tomo, ora, (11, 7, 5), [-1.0, -1.0, -1.0], [1.0, 1.5, 0.5], 3, (0.0, 0.0, 0.0, 0.0),
                0.3, 2.0, 21)


def test_height_prior_parity_euvi_cube(tomo, ora):
    """The 128^3 cube of the EUVI-like inversion ([-1.5, 1.5]^3, heights
    from the Sun's centre), every voxel."""
    _prior_case(tomo, ora, (128, 128, 128), [-1.5, -1.5, -1.5], [1.5, 1.5, 1.5], 1, (0.0, 0.0, 0.0, 0.0),
                1e-2, 0.0, 22)


def test_height_prior_accumulates(tomo, ora):
    g, dg, xf, got = _prior_case(tomo, ora, (9, 8, 7), [-1.0, -1.0, -1.0], [1.0, 1.0, 1.0], 1,
                                 (0.2, 0.1, 0.0, 0.5), 0.8, 0.0, 23)
    base = np.random.default_rng(24).normal(size=dg.cube_shape).astype(np.float32)
    out = to_dev(base)
    tomo.apply_prior(dg, to_dev(xf), 0.8, out=out, accumulate=True, height=(0.2, 0.1, 0.0, 0.5))
    np.testing.assert_allclose(to_host(out), base + got, rtol=1e-6, atol=1e-6)


def _two_instruments(n=16, half=1.3, gains=(0.6, 0.6, 0.6, 2.2, 2.2), masks=True, seed=30):
    """Instrument A: 3 views of 40 x 33 pixels; instrument B: 2 views of
    27 x 45 pixels from other longitudes and distances."""
    va, pa = ts.make_views([10.0, 95.0, 200.0], (40, 33), 3.0, lat=12.0, dist=20.0)
    vb, pb = ts.make_views([40.0, 150.0], (27, 45), 3.4, lat=-20.0, dist=35.0)
    views, npix = np.concatenate([va, vb]), np.concatenate([pa, pb])
    nn, lo, hi = ts.box(n, half)
    g = ts.Geometry(nn, lo, hi, views, npix, gains=None if gains is None else np.array(gains, float))
    if masks:
        rng = np.random.default_rng(seed)
        g.data_mask = (rng.uniform(size=g.nrays) > 0.2).astype(np.uint8)
        g.map_mask = (rng.uniform(size=g.cube_shape()) > 0.15).astype(np.uint8)
    return g


def test_gains_every_pixel_and_voxel(tomo, ora):
    g = _two_instruments()
    rng = np.random.default_rng(31)
    parity_full(tomo, ora, g, rng.uniform(size=g.cube_shape()), rng.normal(size=g.nrays))


def test_negative_and_zero_gains(tomo, ora):
    g = _two_instruments(gains=(1.3, 1.3, 1.3, -0.4, 0.0), masks=False)
    rng = np.random.default_rng(32)
    parity_full(tomo, ora, g, rng.uniform(size=g.cube_shape()), rng.normal(size=g.nrays))


def test_unit_gains_change_no_bit(tomo):
    """Gains of 1 multiply exactly: P and the blocked P^T are bit-identical
    to the geometry without gains."""
    g1 = _two_instruments(gains=(1.0,) * 5)
    g0 = _two_instruments(gains=None)
    d1, d0 = tomo.DeviceGeometry(g1), tomo.DeviceGeometry(g0)
    rng = np.random.default_rng(33)
    x, y = to_dev(rng.uniform(size=g0.cube_shape())), to_dev(rng.normal(size=g0.nrays))
    np.testing.assert_array_equal(to_host(tomo.project(d1, x)), to_host(tomo.project(d0, x)))
    np.testing.assert_array_equal(to_host(tomo.backproject(d1, y, strategy=CODES["blocked"])),
                                  to_host(tomo.backproject(d0, y, strategy=CODES["blocked"])))


def test_batch_with_gains(tomo):
    """Batched P and P^T of a system with gains next to one without equal
    the per-system calls bit for bit."""
    ga, gb = _two_instruments(), _two_instruments(gains=None, seed=34)
    dga, dgb = tomo.DeviceGeometry(ga), tomo.DeviceGeometry(gb)
    rng = np.random.default_rng(35)
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


def test_euvi_two_instruments(tomo, ora):
    """EUVI-like 128^3 (unit sphere masked): one view of each observer at
    512^2 with gains 1 and 1.27, every pixel and voxel."""
    wl = ts.euvi()
    g = wl.geom.subset([0, 1])
    g.gains = np.array([1.0, 1.27])
    y = np.random.default_rng(36).normal(size=g.nrays)
    parity_full(tomo, ora, g, wl.x, y)


def test_euvi_full_size_sampled_gains(tomo, ora):
    """All 28 views with observer B's 14 views at gain 1.27: P on 3000
    sampled pixels (oracle segments times the view's gain)."""
    wl = ts.euvi()
    g = wl.geom.subset(np.arange(wl.geom.nviews))
    g.gains = np.where(np.arange(g.nviews) % 2 == 1, 1.27, 1.0)
    dg = tomo.DeviceGeometry(g)
    img = to_host(tomo.project(dg, to_dev(wl.x)))
    pix = sample_pixels(g, 3000, 37)
    got = np.array([img[flat_index(g, *p)] for p in pix])
    vals, absv = oracle_pixels(ora, g, wl.x, pix)
    gv = np.array([g.gains[p[0]] for p in pix])
    assert_p_close(got, vals * gv, absv * gv, atol=1.27 * length_resolution(g) * np.abs(wl.x).max())


@pytest.mark.parametrize("kind", ["pB", "B"])
def test_thomson_with_gains(tomo, ora, kind):
    """The Thomson operators of a two-instrument coronagraph geometry: each
    instrument's images carry its gain, forward and transpose."""
    nn, lo, hi = ts.box(32, 4.0)
    va, pa = ts.make_views([0.0, 120.0, 240.0], (48, 48), 8.0, lat=7.0)
    vb, pb = ts.make_views([60.0, 180.0], (40, 40), 8.0, lat=-5.0)
    views, npix = np.concatenate([va, vb]), np.concatenate([pa, pb])
    g = ts.Geometry(nn, lo, hi, views, npix, map_mask=ts.sphere_map_mask(nn, lo, hi, 1.0),
                    gains=np.array([1.0, 1.0, 1.0, 0.55, 0.55]))
    u, scale = 0.63, 3.0
    rng = np.random.default_rng(38)
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
    gotb = to_host(tomo.thomson_backproject(dg, to_dev(y), u, kind, scale))
    assert_p_close(gotb, ora.thomson_backproject(g, y, u, kind, scale), ba, rtol=1e-4, what=f"T_{kind}^T",
                   atol=res * float(np.max(np.abs(ba))))


HEIGHT = (0.0, 0.0, 0.0, 0.0)


def _tiny_two_instruments(ora):
    wl = ts.tiny()
    g = wl.geom.subset(np.arange(wl.geom.nviews))
    g.gains = np.where(np.arange(g.nviews) < 4, 0.7, 1.6)
    y = ora.project(g, wl.x).astype(np.float32).astype(np.float64)
    return wl, g, y


def test_cg_height_gains_matches_oracle(tomo, ora):
    """Twenty CG iterations of Eq. srt_multiple_inv with the height-weighted
    prior on the tiny problem (two instruments of 4 views, gains 0.7 and
    1.6): residual history and final x against the FP64 oracle."""
    wl, g, y = _tiny_two_instruments(ora)
    dg = tomo.DeviceGeometry(g)
    x, rep = tomo.cg_solve(dg, to_dev(y), lam_r=wl.lam_r, max_iter=20, height=HEIGHT)
    xg = to_host(x)
    xo, ho = ora.cg(ora.normal_operator(g, wl.lam_r, height=HEIGHT), ora.rhs(g, y), n_iter=20)
    assert rep["iters"] == 20 and rep["status"] == 0
    np.testing.assert_allclose(rep["history"], ho, rtol=2e-4)
    assert np.linalg.norm(xg - xo) <= 1e-4 * np.linalg.norm(xo)
    assert abs(rep["true_rel_res"] - rep["rel_res"]) <= 1e-3 * rep["rel_res"] + 1e-6


def test_cg_masked_frames_height(tomo, ora):
    """Three frames, map mask, temporal prior and the height-weighted
    spatial prior with an offset: 15 iterations."""
    wl = ts.tiny()
    g0 = wl.geom
    vf = (np.arange(g0.nviews) % 3).astype(np.int32)
    mm = ts.sphere_map_mask(g0.n, g0.lo, g0.hi, 0.6)
    g = ts.Geometry(g0.n, g0.lo, g0.hi, g0.views, g0.npix, vf, 3, None, mm,
                    gains=np.linspace(0.8, 1.4, g0.nviews))
    x = np.stack([wl.x * (1 + 0.1 * f) for f in range(3)])
    y = ora.project(g, x).astype(np.float32).astype(np.float64)
    h = (0.1, -0.05, 0.0, -0.5)
    dg = tomo.DeviceGeometry(g)
    xg, rep = tomo.cg_solve(dg, to_dev(y), lam_r=1e-2, lam_t=10.0, max_iter=15, height=h)
    xg = to_host(xg)
    xo, ho = ora.cg(ora.normal_operator(g, 1e-2, 10.0, height=h), ora.rhs(g, y), n_iter=15)
    np.testing.assert_allclose(rep["history"], ho, rtol=2e-4)
    assert np.linalg.norm(xg - xo) <= 1e-4 * np.linalg.norm(xo)
    assert np.all(xg[:, mm == 0] == 0.0)


def test_batch_cg_height_gains(tomo, ora):
    """The batched, graph-captured CG with one height-weighted system with
    gains next to a plain one: each against its own oracle solve."""
    wl, g, y = _tiny_two_instruments(ora)
    g2 = wl.geom
    y2 = ora.project(g2, wl.x).astype(np.float32).astype(np.float64)
    dga, dgb = tomo.DeviceGeometry(g), tomo.DeviceGeometry(g2)
    batch = tomo.Batch([dga, dgb])
    try:
        xs, reps = batch.cg_solve([to_dev(y), to_dev(y2)], lam_r=wl.lam_r, max_iter=20, use_graph=True,
                                  check_every=5, heights=[HEIGHT, None])
    finally:
        batch.close()
    for xg, rep, gg, yy, hh in zip(xs, reps, (g, g2), (y, y2), (HEIGHT, None)):
        xo, ho = ora.cg(ora.normal_operator(gg, wl.lam_r, height=hh), ora.rhs(gg, yy), n_iter=20)
        np.testing.assert_allclose(rep["history"], ho, rtol=2e-4)
        xh = to_host(xg)
        assert np.linalg.norm(xh - xo) <= 1e-4 * np.linalg.norm(xo)


def test_two_instruments_recover_the_map(tomo, ora):
    """Noise-free data of two instruments (gains 0.6 and 2.2) on a 3^3 cube
    seen by 5 views: with the gains in the geometry, CG run to a tight
    residual recovers the map, which the same data without gains do not."""
    va, pa = ts.make_views([10.0, 95.0, 200.0], (9, 7), 3.0, lat=12.0, dist=20.0)
    vb, pb = ts.make_views([40.0, 150.0], (6, 11), 3.4, lat=-20.0, dist=35.0)
    views, npix = np.concatenate([va, vb]), np.concatenate([pa, pb])
    nn, lo, hi = ts.box(3, 1.0)
    g = ts.Geometry(nn, lo, hi, views, npix, gains=np.array([0.6, 0.6, 0.6, 2.2, 2.2]))
    e = np.random.default_rng(11).uniform(0.5, 2.0, size=g.cube_shape())
    y = ora.project(g, e)
    # the normal matrix has condition number ~27: a residual of 1e-5 leaves
    # an error below ~3e-4 of the map
    x, rep = tomo.cg_solve(tomo.DeviceGeometry(g), to_dev(y), lam_r=0.0, max_iter=200, rtol=1e-5)
    assert rep["status"] == 0
    np.testing.assert_allclose(to_host(x), e, rtol=2e-3)
    g1 = ts.Geometry(nn, lo, hi, views, npix)
    x1, _ = tomo.cg_solve(tomo.DeviceGeometry(g1), to_dev(y), lam_r=0.0, max_iter=200, rtol=1e-5)
    assert np.abs(to_host(x1) - e).max() > 0.1
