"""GPU parity of P and P^T (through the C ABI) against the FP64 oracle."""
import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import (CODES, assert_p_close, flat_index, length_resolution, need_gpu, oracle_pixels,
                         parity_full as _parity_full, sample_pixels, to_dev, to_host)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tomo():
    return need_gpu()


def test_tiny_projection_and_transpose(tomo, ora):
    wl = ts.tiny()
    y = np.random.default_rng(1).normal(size=wl.geom.nrays)
    _parity_full(tomo, ora, wl.geom, wl.x, y)


def test_masks(tomo, ora):
    wl = ts.tiny()
    g = wl.geom
    rng = np.random.default_rng(7)
    dm = (rng.uniform(size=g.nrays) > 0.3).astype(np.uint8)
    mm = (rng.uniform(size=g.cube_shape()) > 0.2).astype(np.uint8)
    gm = ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, data_mask=dm, map_mask=mm)
    _parity_full(tomo, ora, gm, wl.x, rng.normal(size=g.nrays))


def test_frames(tomo, ora):
    wl = ts.tiny()
    g = wl.geom
    vf = (np.arange(g.nviews) % 3).astype(np.int32)
    gf = ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, vf, 3)
    x = np.stack([wl.x * (f + 1) for f in range(3)])
    _parity_full(tomo, ora, gf, x, np.random.default_rng(2).normal(size=g.nrays))


def test_ragged_views_and_box(tomo, ora):
    """Non-cubic grid in an off-centre box, views whose sizes leave partial
    16x16 tiles, a one-pixel view, and an observer inside the box."""
    n, lo, hi = (20, 13, 9), np.array([-1.3, -0.6, -0.9]), np.array([1.7, 1.1, 0.45])
    rows, pix = [], []
    for lon, (nc, nr), fov in [(10.0, (37, 23), 3.0), (123.0, (5, 70), 2.5), (250.0, (1, 1), 1.0)]:
        r, p = ts.pinhole_view(ts.observer(lon, 12.0, 40.0), npix=(nc, nr), fov=fov)
        rows.append(r)
        pix.append([nc, nr])
    r, p = ts.pinhole_view(np.array([0.2, 0.1, -0.1]), target=(1.0, 0.3, 0.2), npix=(24, 24), fov=8.0)
    rows.append(r)
    pix.append([24, 24])
    g = ts.Geometry(n, lo, hi, np.array(rows), np.array(pix, dtype=np.int32))
    x = np.random.default_rng(3).uniform(size=g.cube_shape())
    _parity_full(tomo, ora, g, x, np.random.default_rng(4).normal(size=g.nrays))


def test_euvi_two_views_full(tomo, ora):
    """EUVI-like 128^3 cube with the unit sphere masked, two of the 28 views at
    512x512: every pixel and every voxel compared."""
    wl = ts.euvi()
    g = wl.geom.subset([0, 13])
    y = np.random.default_rng(5).normal(size=g.nrays)
    _parity_full(tomo, ora, g, wl.x, y)


def test_euvi_full_size_sampled(tomo, ora):
    """All 28 views at 512x512 in one launch (the benchmark's configuration):
    P compared on 4000 sampled pixels, P^T on an image that is non-zero on
    300 sampled pixels only (so the oracle needs only those rays)."""
    wl = ts.euvi()
    g = wl.geom
    dg = tomo.DeviceGeometry(g)
    img = to_host(tomo.project(dg, to_dev(wl.x)))
    pix = sample_pixels(g, 4000, 11)
    val, absv = oracle_pixels(ora, g, wl.x, pix)
    got = np.array([img[flat_index(g, *p)] for p in pix])
    assert_p_close(got, val, absv)
    sel = sample_pixels(g, 300, 12)
    y = np.zeros(g.nrays)
    rng = np.random.default_rng(13)
    for p in sel:
        y[flat_index(g, *p)] = rng.normal()
    bp = to_host(tomo.backproject(dg, to_dev(y)))
    assert tomo.binning_spills(dg) == 0
    # oracle P^T from the selected rays only
    ref = np.zeros(g.nvox)
    refa = np.zeros(g.nvox)
    for p in sel:
        yv = y[flat_index(g, *p)]
        d = ora.pixel_direction(g.views[p[0]], g.npix[p[0]], p[1], p[2])
        idx, ln, _ = ora.trace_ray(g.n, g.lo, g.hi, g.views[p[0]][0:3], d)
        keep = g.map_mask.reshape(-1)[idx] == 1
        np.add.at(ref, idx[keep], ln[keep] * yv)
        np.add.at(refa, idx[keep], ln[keep] * abs(yv))
    assert_p_close(bp, ref, refa, rtol=1e-4, what="P^T",
                   atol=length_resolution(g) * np.abs(y).max())


def _dyadic_geometry():
    """Box [-1, 1]^3, N = 16; an observer looking along +x with axis-aligned
    detector vectors and cdelt 1/64, so pixel offsets of 0, +-1, +-2, +-4, +-8
    from crpix give directions whose components are powers of two."""
    row = np.concatenate([[-3.0, 0.25, -0.375], [1, 0, 0], [0, 1, 0], [0, 0, 1],
                          [1 / 64, 1 / 64], [8.0, 8.0]])
    row2 = np.concatenate([[0.125, -2.5, 0.0625], [0, 1, 0], [0, 0, 1], [1, 0, 0],
                           [1 / 16, 1 / 32], [8.0, 8.0]])
    views = np.array([row, row2])
    return ts.Geometry((16, 16, 16), np.full(3, -1.0), np.full(3, 1.0), views,
                       np.array([[17, 17], [17, 17]], dtype=np.int32))


def test_trace_dyadic_bit_exact(tomo, ora):
    """On dyadic rays every crossing is exact on both sides: voxel index
    sequences and parametric segment lengths agree bit for bit, and lengths
    to the last bit of |d|."""
    g = _dyadic_geometry()
    dg = tomo.DeviceGeometry(g)
    offs = [0, 1, -1, 2, -2, 4, -4, 8, -8]
    checked = 0
    for v in range(2):
        for dc in offs:
            for dr in offs:
                col, row = 8 + dc, 8 + dr
                gi, gl, gp = tomo.trace_ray(dg, v, col, row)
                d = ora.pixel_direction(g.views[v], g.npix[v], col, row)
                oi, ol, ot = ora.trace_ray(g.n, g.lo, g.hi, g.views[v][0:3], d)
                assert gi.tolist() == oi.tolist(), (v, col, row)
                if len(ot) > 1:  # parametric lengths between interior boundaries
                    assert np.array_equal(gp[:-1], np.diff(ot)), (v, col, row)
                np.testing.assert_allclose(gl, ol, rtol=4e-16, atol=0)
                checked += len(gi)
    assert checked > 500


def test_trace_generic_rays(tomo, ora):
    """Generic rays of the tiny geometry.  Its 45-degree views make x and y
    crossings coincide to within an ulp (cos 45 and sin 45 differ in the last
    bit), and the two sides may order such a near-tie differently with a
    segment of ~1e-16 in between: after dropping segments shorter than 1e-12
    of the box, the voxel sequences must agree exactly, and the length inside
    every voxel to 1e-12."""
    wl = ts.tiny()
    g = wl.geom
    dg = tomo.DeviceGeometry(g)
    tiny = 1e-12 * 3.0
    for v, col, row in sample_pixels(g, 300, 3):
        gi, gl, _ = tomo.trace_ray(dg, v, col, row)
        d = ora.pixel_direction(g.views[v], g.npix[v], col, row)
        oi, ol, _ = ora.trace_ray(g.n, g.lo, g.hi, g.views[v][0:3], d)
        assert gi[gl > tiny].tolist() == oi[ol > tiny].tolist(), (v, col, row)
        rg, ro = np.zeros(g.nvox), np.zeros(g.nvox)
        np.add.at(rg, gi, gl)
        np.add.at(ro, oi, ol)
        np.testing.assert_allclose(rg, ro, rtol=0, atol=1e-12)


def test_crossing_counts(tomo, ora):
    wl = ts.tiny()
    dg = tomo.DeviceGeometry(wl.geom)
    assert tomo.count_crossings(dg) == ora.count_crossings(wl.geom)
    g2 = ts.euvi().geom.subset([0, 5])
    c_gpu = tomo.count_crossings(tomo.DeviceGeometry(g2))
    c_ora = ora.count_crossings(g2)
    # near-ties (crossings closer than ~1e-15 of the chord) may merge on one side
    assert abs(c_gpu - c_ora) <= 1e-8 * c_ora + 2


def test_adjoint_identity(tomo):
    """<P x, y> = <x, P^T y> for 100 random pairs (FP32 data, FP64 sums)."""
    import torch

    wl = ts.tiny()
    dg = tomo.DeviceGeometry(wl.geom)
    worst = 0.0
    for seed in range(500, 600):
        x, y = ts.random_pair(wl.geom.nvox, wl.geom.nrays, seed)
        xd, yd = to_dev(x), to_dev(y)
        px = tomo.project(dg, xd).double()
        pty = tomo.backproject(dg, yd).double()
        lhs = float(torch.dot(px, yd.double()))
        rhs = float(torch.dot(xd.double().ravel(), pty.ravel()))
        scale = float(torch.linalg.norm(px)) * float(np.linalg.norm(y))
        worst = max(worst, abs(lhs - rhs) / scale)
    assert worst <= 1e-5


@pytest.fixture
def tuning(tomo):
    """Restores the process-wide tuning after a test changes it."""
    old = tomo.get_tuning()
    yield tomo
    tomo.set_tuning(**old)


@pytest.mark.parametrize("block,splits", [((4, 4, 4), 1), ((5, 3, 7), 3), ((32, 2, 9), 0), ((16, 16, 16), 8)])
def test_blocked_shapes(tuning, ora, block, splits):
    """The blocked P^T with small, ragged and flat voxel blocks and several
    owners per block, on the tiny, masked and multi-frame geometries."""
    tomo = tuning
    tomo.set_tuning(bp_block=block, bp_splits=splits)
    wl = ts.tiny()
    g = wl.geom
    rng = np.random.default_rng(21)
    _parity_full(tomo, ora, g, wl.x, rng.normal(size=g.nrays), strategies=["blocked"])
    dm = (rng.uniform(size=g.nrays) > 0.3).astype(np.uint8)
    mm = (rng.uniform(size=g.cube_shape()) > 0.2).astype(np.uint8)
    vf = (np.arange(g.nviews) % 3).astype(np.int32)
    gm = ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, vf, 3, data_mask=dm, map_mask=mm)
    x3 = np.stack([wl.x * (f + 1) for f in range(3)])
    _parity_full(tomo, ora, gm, x3, rng.normal(size=g.nrays), strategies=["blocked"])


def test_blocked_footprint_rows_drop_no_ray(tuning):
    """With one owner per block the fixed-point bins sum every voxel exactly,
    so the blocked P^T cannot depend on the block shape.  Flat blocks seen
    from the ecliptic walk one column interval per footprint row; 8x8x64
    blocks there have footprints taller than the row table and walk whole
    rectangles (and the other way round from the poles).  Any ray an
    interval dropped would change some voxel: the outputs must agree bit for
    bit on aligned, close, odd-sized, off-ecliptic and random views."""
    import torch

    tomo = tuning
    rng = np.random.default_rng(41)
    rows, pix = [], []
    specs = [(ts.observer(lon), (0.0, 0.0, 0.0), (128, 128), 3.2) for lon in (0.0, 45.0, 90.0)]
    specs += [(ts.observer(20.0, 0.0, 3.0), (0.0, 0.0, 0.0), (97, 61), 3.0)]
    specs += [(ts.observer(rng.uniform(0, 360), lat), (0.0, 0.0, 0.0), (120, 100), 3.2) for lat in (30.0, 60.0, 89.0)]
    for _ in range(3):
        d = rng.normal(size=3)
        specs.append((d / np.linalg.norm(d) * rng.uniform(2.5, 40.0), tuple(rng.uniform(-0.3, 0.3, 3)),
                      (int(rng.integers(40, 160)), int(rng.integers(40, 160))), rng.uniform(1.0, 5.0)))
    for obs, target, npix, fov in specs:
        r, p = ts.pinhole_view(np.asarray(obs, dtype=np.float64), target=target, npix=npix, fov=fov)
        rows.append(r)
        pix.append(p)
    g = ts.Geometry((64, 64, 64), np.full(3, -1.5), np.full(3, 1.5), np.array(rows), np.array(pix, np.int32))
    dg = tomo.DeviceGeometry(g)
    y = torch.as_tensor(rng.normal(size=g.nrays).astype(np.float32)).cuda()
    outs = {}
    for block in ((8, 8, 64), (64, 32, 2), (32, 32, 4), (16, 16, 16), (64, 8, 16)):
        tomo.set_tuning(bp_block=block, bp_splits=1)
        outs[block] = tomo.backproject(dg, y, strategy=tomo.BP_BLOCKED).clone()
    ref = outs[(8, 8, 64)]
    assert float(ref.abs().max()) > 0
    for block, out in outs.items():
        assert torch.equal(out, ref), block


@pytest.mark.parametrize("block", [(4, 4, 4), (5, 3, 7)])
def test_blocked_one_hot_rays_match_the_walk(tuning, block):
    """P^T of a one-hot image through the blocked strategy is that ray's
    segment list: the same voxels as the full walk (tomo_trace_ray) and the
    same lengths to FP32 rounding, although every ray is walked piecewise
    through many small blocks."""
    import torch

    tomo = tuning
    tomo.set_tuning(bp_block=block, bp_splits=1)
    wl = ts.tiny()
    g = wl.geom
    dg = tomo.DeviceGeometry(g)
    y = torch.zeros(g.nrays, dtype=torch.float32, device="cuda")
    checked = 0
    for v, col, row in sample_pixels(g, 120, 31):
        gi, gl, _ = tomo.trace_ray(dg, v, col, row)
        k = flat_index(g, v, col, row)
        y.zero_()
        y[k] = 1.0
        bp = to_host(tomo.backproject(dg, y, strategy=tomo.BP_BLOCKED)).reshape(-1)
        ref = np.zeros(g.nvox)
        np.add.at(ref, gi, gl)
        # near-tie segments of ~1e-16 fall below the fixed-point quantum
        # (~1e-15 here) and may vanish; everything else must be there
        got = set(np.flatnonzero(bp).tolist())
        assert set(gi[gl > 3e-12].tolist()) <= got <= set(gi.tolist()), (v, col, row)
        np.testing.assert_allclose(bp, ref, rtol=2.0 ** -23, atol=1e-12)
        checked += len(gi)
    assert checked > 1000


def test_blocked_is_deterministic(tomo):
    import torch

    wl = ts.euvi()
    g = wl.geom.subset([0, 3, 7])
    dg = tomo.DeviceGeometry(g)
    y = to_dev(np.random.default_rng(8).normal(size=g.nrays))
    a = tomo.backproject(dg, y, strategy=tomo.BP_BLOCKED)
    b = tomo.backproject(dg, y, strategy=tomo.BP_BLOCKED)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def _mixed_geometry(rng, n=64, with_masks=False):
    """Views from the ecliptic, the poles, close up and at random, over an
    n^3 cube; optionally random data and map masks."""
    rows, pix = [], []
    specs = [(ts.observer(lon), (0.0, 0.0, 0.0), (128, 128), 3.2) for lon in (10.0, 45.0, 100.0)]
    specs += [(ts.observer(20.0, 0.0, 3.0), (0.0, 0.0, 0.0), (97, 61), 3.0)]
    specs += [(ts.observer(rng.uniform(0, 360), lat), (0.0, 0.0, 0.0), (120, 100), 3.2) for lat in (30.0, 89.0)]
    for _ in range(2):
        d = rng.normal(size=3)
        specs.append((d / np.linalg.norm(d) * rng.uniform(2.5, 40.0), tuple(rng.uniform(-0.3, 0.3, 3)),
                      (int(rng.integers(40, 160)), int(rng.integers(40, 160))), rng.uniform(1.0, 5.0)))
    for obs, target, npix, fov in specs:
        r, p = ts.pinhole_view(np.asarray(obs, dtype=np.float64), target=target, npix=npix, fov=fov)
        rows.append(r)
        pix.append(p)
    g = ts.Geometry((n, n, n), np.full(3, -1.5), np.full(3, 1.5), np.array(rows), np.array(pix, np.int32))
    if with_masks:
        g.data_mask = (rng.uniform(size=g.nrays) > 0.35).astype(np.uint8)
        g.map_mask = (rng.uniform(size=g.cube_shape()) > 0.1).astype(np.uint8)
    return g


@pytest.mark.parametrize("masks", [False, True])
def test_blocked_workgroup_sizes(tuning, ora, masks):
    """The blocked P^T for workgroups of 256, 512 and 1024 lanes, with the
    larger blocks those own (up to 16384 voxels of LDS bins), one owner per
    block: every output bit equal whatever the shape (the fixed-point sums
    are exact), and the whole operator against the oracle.  With a data mask
    the passes take the kept pixels of each footprint row only."""
    import torch

    tomo = tuning
    rng = np.random.default_rng(51 + int(masks))
    g = _mixed_geometry(rng, with_masks=masks)
    dg = tomo.DeviceGeometry(g)
    y = rng.normal(size=g.nrays).astype(np.float32).astype(np.float64)
    yd = to_dev(y)
    outs = {}
    for nt, block in ((256, (64, 32, 2)), (256, (16, 16, 16)), (512, (64, 64, 2)), (512, (32, 32, 8)),
                      (1024, (128, 64, 2)), (1024, (32, 32, 16)), (1024, (64, 64, 4))):
        tomo.set_tuning(bp_threads=nt, bp_block=block, bp_splits=1)
        outs[(nt, block)] = tomo.backproject(dg, yd, strategy=tomo.BP_BLOCKED).clone()
        assert tomo.binning_spills(dg) == 0
    ref = outs[(256, (64, 32, 2))]
    for key, out in outs.items():
        assert torch.equal(out, ref), key
    res = length_resolution(g)
    assert_p_close(to_host(ref), ora.backproject(g, y), ora.backproject(g, np.abs(y)), rtol=1e-4,
                   what="P^T", atol=res * np.abs(y).max())


@pytest.mark.parametrize("layout", [2, 3, 4])
def test_bricked_projection_equals_linear(tuning, ora, layout):
    """P from a bricked copy of the cube (bricks of 4, 8 and 16 voxels a
    side) walks the same segments in the same order as from the x-fastest
    cube: the same bits, on ragged boxes whose sides are not multiples of
    the brick, with masks, frames and the obstacle."""
    import torch

    tomo = tuning
    rng = np.random.default_rng(60 + layout)
    g1 = _mixed_geometry(rng, n=37, with_masks=True)
    wl = ts.tiny()
    g0 = wl.geom
    vf = (np.arange(g0.nviews) % 3).astype(np.int32)
    g2 = ts.Geometry(g0.n, g0.lo, g0.hi, g0.views, g0.npix, vf, 3,
                     map_mask=(rng.uniform(size=g0.cube_shape()) > 0.2).astype(np.uint8))
    g3 = ts.Geometry((23, 41, 19), np.array([-1.3, -1.5, -0.9]), np.array([1.4, 1.2, 1.1]), g0.views, g0.npix,
                     obstacle=np.array([0.1, 0.0, -0.1, 0.7]))
    for g in (g1, g2, g3):
        dg = tomo.DeviceGeometry(g)
        x = to_dev(rng.uniform(size=g.cube_shape()))
        tomo.set_tuning(p_layout=0)
        ref = tomo.project(dg, x).clone()
        tomo.set_tuning(p_layout=layout)
        got = tomo.project(dg, x)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)
        assert float(ref.abs().max()) > 0
    # and the bricked P agrees with the oracle on the masked geometry
    dg = tomo.DeviceGeometry(g1)
    x = rng.uniform(size=g1.cube_shape())
    res = length_resolution(g1)
    img = to_host(tomo.project(dg, to_dev(x)))
    assert_p_close(img, ora.project(g1, x), ora.project(g1, np.abs(x * g1.map_mask)), atol=res * np.abs(x).max())
