"""Pins of the oracle's obstacle variant: every line of sight ends where it
enters the opaque sphere (the photosphere; Sec. "Solar Tomography", the
projector's obstacle variant in Sec. "Fast Parallelized Projector", and the
integration stopping at the photosphere in Sec. "Performance").  Checked
against chords derived by hand, the per-voxel brute force, dense sampling
along the ray, and the adjoint identity."""
import numpy as np
import pytest

import tomo_synth as ts

N6 = np.array([6, 6, 6], dtype=np.int32)
LO, HI = np.full(3, -1.5), np.full(3, 1.5)
SUN = np.array([0.0, 0.0, 0.0, 1.0])


def _total(ora, o, d, obstacle=SUN, n=N6, lo=LO, hi=HI):
    _, ln, _ = ora.trace_ray(n, lo, hi, np.asarray(o, float), np.asarray(d, float), obstacle)
    return float(np.sum(ln))


def test_hand_chords(ora):
    # along +x at height r from the axis through the centre: from the box face
    # x = -1.5 to the sphere at x = -sqrt(1 - r^2)
    assert _total(ora, (-5, 0, 0), (1, 0, 0)) == pytest.approx(0.5, abs=1e-14)
    assert _total(ora, (-5, 0.6, 0), (1, 0, 0)) == pytest.approx(0.7, abs=1e-14)
    assert _total(ora, (-5, 0.6, 0.48), (1, 0, 0)) == pytest.approx(0.86, abs=1e-14)
    # a longer direction vector gives the same geometric length
    assert _total(ora, (-5, 0.6, 0.48), (2, 0, 0)) == pytest.approx(0.86, abs=1e-14)
    # tangent and passing lines are not blocked: the whole chord
    assert _total(ora, (-5, 1.0, 0), (1, 0, 0)) == pytest.approx(3.0, abs=1e-14)
    assert _total(ora, (-5, 0.8, 0.8), (1, 0, 0)) == pytest.approx(3.0, abs=1e-14)
    # diagonal through the centre: enters the box at t with x = y = -1.5
    # (distance 1.5 sqrt 2 from the axis origin) and stops at distance 1
    assert _total(ora, (-5, -5, 0), (1, 1, 0)) == pytest.approx(1.5 * np.sqrt(2) - 1.0, abs=1e-13)


def test_hand_segments(ora):
    """Voxels of side 0.5: the ray at (y, z) = (0.6, 0.48) crosses x = -1.5
    .. -1 whole (0.5) and stops at x = -0.64 inside the next voxel (0.36)."""
    idx, ln, _ = ora.trace_ray(N6, LO, HI, np.array([-5.0, 0.6, 0.48]), np.array([1.0, 0, 0]), SUN)
    j, k = int((0.6 + 1.5) / 0.5), int((0.48 + 1.5) / 0.5)
    assert list(idx) == [(k * 6 + j) * 6 + 0, (k * 6 + j) * 6 + 1]
    np.testing.assert_allclose(ln, [0.5, 0.36], atol=1e-14)


def test_observer_inside_or_behind(ora):
    # inside the sphere: nothing is seen, whatever the direction
    assert _total(ora, (0.2, 0, 0), (1, 0, 0)) == 0.0
    assert _total(ora, (0.0, 0.5, 0), (0, -1, 0)) == 0.0
    # on the sphere: nothing is seen either
    assert _total(ora, (1.0, 0, 0), (1, 0, 0)) == 0.0
    # outside the sphere, moving away from it: from x = 1.2 to the face
    assert _total(ora, (1.2, 0, 0), (1, 0, 0)) == pytest.approx(0.3, abs=1e-14)
    # the sphere blocks the line before it reaches the box
    far = np.array([-3.0, 0.5, 0.5, 1.0])
    assert _total(ora, (-6, 0.5, 0.5), (1, 0, 0), far, np.array([4, 4, 4], np.int32),
                  np.zeros(3), np.ones(3)) == 0.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rows_match_the_brute_force(ora, seed):
    """Siddon with the obstacle equals the per-voxel slab clip cut at the
    sphere, on random rays that start outside, pass beside, or graze."""
    rng = np.random.default_rng(seed)
    n = np.array([5, 7, 6], dtype=np.int32)
    lo, hi = np.array([-1.3, -1.6, -1.2]), np.array([1.4, 1.2, 1.5])
    sph = np.array([0.1, -0.2, 0.05, 0.9])
    for _ in range(200):
        o = rng.normal(size=3)
        o *= rng.uniform(1.5, 6.0) / np.linalg.norm(o)
        d = rng.uniform(-0.6, 0.6, size=3) - o / np.linalg.norm(o)
        idx, ln, _ = ora.trace_ray(n, lo, hi, o, d, sph)
        row = np.zeros(int(np.prod(n)))
        np.add.at(row, idx, ln)
        np.testing.assert_allclose(row, ora.ray_row_bruteforce(n, lo, hi, o, d, sph), atol=1e-12)


def _near_views():
    """The tiny cube seen from 4 R_sun by 6 views of 24 x 20 pixels over a
    3.2 R_sun field: the sphere hides part of the box, and many lines of
    sight pass beside it."""
    n, lo, hi = ts.box(16, 1.5)
    views, npix = ts.make_views([0.0, 50.0, 110.0, 190.0, 250.0, 320.0], (24, 20), 3.2, lat=15.0, dist=4.0)
    return ts.Geometry(n, lo, hi, views, npix, obstacle=SUN.copy())


def test_constant_cube_by_dense_sampling(ora):
    """P of a cube of ones is the length of the line of sight inside the box
    and in front of the sphere; that length is measured here by sampling the
    line at 2e5 points (independent of any formula)."""
    go = _near_views()
    views = go.views
    img = ora.project(go, np.ones(go.cube_shape()))
    rng = np.random.default_rng(5)
    t = (np.arange(200000) + 0.5) / 200000 * 12.0
    for _ in range(40):
        v = int(rng.integers(go.nviews))
        col, row = (int(rng.integers(k)) for k in go.npix[v])
        o = views[v, 0:3]
        d = ora.pixel_direction(views[v], go.npix[v], col, row)
        p = o[None, :] + t[:, None] * d[None, :]
        inside = np.all((p >= go.lo) & (p < go.hi), axis=1)
        blocked = np.cumsum(np.sum(p * p, axis=1) < 1.0) > 0
        est = np.count_nonzero(inside & ~blocked) * (12.0 / 200000) * np.linalg.norm(d)
        k = go.view_offsets()[v] + row * go.npix[v][0] + col
        assert abs(img[k] - est) < 2e-4 * np.linalg.norm(d) + 1e-12


def test_adjoint_and_counts(ora):
    go = _near_views()
    g, views = go, go.views
    rng = np.random.default_rng(6)
    x, y = rng.normal(size=go.cube_shape()), rng.normal(size=go.nrays)
    lhs = float(np.dot(ora.project(go, x), y))
    rhs = float(np.sum(x * ora.backproject(go, y)))
    assert lhs == pytest.approx(rhs, rel=1e-12)
    free = ts.Geometry(g.n, g.lo, g.hi, views, g.npix)
    assert 0 < ora.count_crossings(go) < ora.count_crossings(free)
    # a sphere that no line of sight enters changes nothing
    away = ts.Geometry(g.n, g.lo, g.hi, views, g.npix, obstacle=np.array([50.0, 50.0, 50.0, 1.0]))
    np.testing.assert_array_equal(ora.project(away, x), ora.project(free, x))
