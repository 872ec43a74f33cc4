"""Pins of the oracle's height-weighted prior R D^T D R (Eq. srt_inversion:
R the diagonal of voxel heights) and of the per-instrument gains of the
multi-spacecraft operator (Eq. two_spacecraft, Eq. lin2space,
Eq. srt_multiple_inv): hand values, a brute-force D and R built by
enumerating neighbour pairs, the prior's null space, the chord of a uniform
box times each view's gain, adjointness, the gradient of the criterion, and
the recovery of a map from noise-free data of two instruments with
different gains."""
import numpy as np
import pytest

import tomo_synth as ts


def _line_geom(lo, hi, n):
    views, npix = ts.make_views([0.0], (2, 2), 1.0, dist=30.0)
    return ts.Geometry(n, np.array(lo, float), np.array(hi, float), views, npix)


def test_height_hand_values(ora):
    """Two voxels on [0, 2] x [-1/2, 1/2]^2, heights from the origin 1/2 and
    3/2.  For x = (1, 1): D R x = 3/2 - 1/2 = 1 and R D^T (1) = (-1/2, 3/2).
    With offset -1 the heights are -1/2 and 1/2: D R x = 1 again and
    R D^T (1) = (1/2, 1/2)."""
    g = _line_geom([0.0, -0.5, -0.5], [2.0, 0.5, 0.5], (2, 1, 1))
    h = ora.voxel_heights(g, (0.0, 0.0, 0.0, 0.0))
    np.testing.assert_allclose(h.reshape(-1), [0.5, 1.5], rtol=1e-15)
    x = np.ones((1, 1, 2))
    np.testing.assert_allclose(ora.height_prior(x, h).reshape(-1), [-0.5, 1.5], rtol=1e-15)
    h1 = ora.voxel_heights(g, (0.0, 0.0, 0.0, -1.0))
    np.testing.assert_allclose(ora.height_prior(x, h1).reshape(-1), [0.5, 0.5], rtol=1e-15)


def test_height_is_the_distance_to_the_centre(ora):
    """A voxel centred at (3, 4, 0) is 5 from the origin and sqrt(9 + 16 + 1)
    = sqrt(26) from (0, 0, 1); the offset adds to the distance."""
    g = _line_geom([2.5, 3.5, -0.5], [3.5, 4.5, 0.5], (1, 1, 1))
    assert float(ora.voxel_heights(g, (0, 0, 0, 0)).reshape(-1)[0]) == pytest.approx(5.0, rel=1e-15)
    assert float(ora.voxel_heights(g, (0, 0, 1, 0)).reshape(-1)[0]) == pytest.approx(np.sqrt(26.0), rel=1e-15)
    assert float(ora.voxel_heights(g, (0, 0, 0, 0.25)).reshape(-1)[0]) == pytest.approx(5.25, rel=1e-15)


def _pairs(n):
    """Neighbour pairs (a, b) of an nx x ny x nz grid, b = a + one step
    along x, y or z, flat index (k ny + j) nx + i."""
    nx, ny, nz = n
    out = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                a = (k * ny + j) * nx + i
                if i + 1 < nx:
                    out.append((a, a + 1))
                if j + 1 < ny:
                    out.append((a, a + nx))
                if k + 1 < nz:
                    out.append((a, a + nx * ny))
    return out


def _heights_by_loops(g, c, off):
    nx, ny, nz = g.n
    d = (g.hi - g.lo) / np.array(g.n, float)
    h = np.zeros(nx * ny * nz)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                p = g.lo + (np.array([i, j, k]) + 0.5) * d - np.asarray(c, float)
                h[(k * ny + j) * nx + i] = np.sqrt(p @ p) + off
    return h


@pytest.mark.parametrize("height", [(0.0, 0.0, 0.0, 0.0), (0.4, -0.9, 1.3, -1.0)])
def test_height_prior_against_explicit_matrices(ora, height):
    """D from an explicit pair list, R from per-voxel loops, on a 3 x 4 x 5
    grid in an uneven box; compare R D^T D R x and ||D R x||^2."""
    n = (3, 4, 5)
    g = _line_geom([-1.2, -0.7, -2.0], [1.5, 1.9, 0.6], n)
    pairs = _pairs(n)
    nv = 60
    D = np.zeros((len(pairs), nv))
    for r, (a, b) in enumerate(pairs):
        D[r, a], D[r, b] = -1.0, 1.0
    hv = _heights_by_loops(g, height[:3], height[3])
    R = np.diag(hv)
    x = np.random.default_rng(5).normal(size=(5, 4, 3))
    h = ora.voxel_heights(g, height)
    np.testing.assert_allclose(h.reshape(-1), hv, rtol=1e-14)
    want = R @ D.T @ D @ R @ x.reshape(-1)
    np.testing.assert_allclose(ora.height_prior(x, h).reshape(-1), want, rtol=1e-12, atol=1e-12)
    e = float(x.reshape(-1) @ ora.height_prior(x, h).reshape(-1))
    assert e == pytest.approx(float(np.sum((D @ R @ x.reshape(-1)) ** 2)), rel=1e-12)


def test_height_prior_null_space(ora):
    """x = c / h makes R x constant, so the weighted prior vanishes while the
    plain one does not (heights positive: centre outside the box)."""
    g = _line_geom([1.0, 1.0, 1.0], [3.0, 2.0, 4.0], (6, 5, 7))
    h = ora.voxel_heights(g, (0.0, 0.0, 0.0, 0.0))
    assert np.all(h > 0)
    x = 2.5 / h
    np.testing.assert_allclose(ora.height_prior(x, h), 0.0, atol=1e-13)
    assert np.abs(ora.laplacian6(x)).max() > 1e-3


def test_height_prior_per_frame(ora):
    """With time frames the same R weighs every frame."""
    g = _line_geom([-1.0, -1.0, -1.0], [1.0, 1.0, 1.0], (4, 3, 5))
    h = ora.voxel_heights(g, (0.1, 0.2, 0.3, 0.0))
    x = np.random.default_rng(6).normal(size=(3, 5, 3, 4))
    got = ora.height_prior(x, h)
    for f in range(3):
        np.testing.assert_allclose(got[f], ora.height_prior(x[f], h), rtol=1e-15)


def _chord(lo, hi, o, d):
    """Length of the half-line o + t d inside the box (slab clip)."""
    t0, t1 = 0.0, np.inf
    for a in range(3):
        if d[a] == 0.0:
            if not lo[a] <= o[a] <= hi[a]:
                return 0.0
            continue
        ta, tb = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return max(t1 - t0, 0.0) * float(np.linalg.norm(d))


def _two_instruments():
    """Instrument A: 3 views of 9 x 7 pixels; instrument B: 2 views of
    6 x 11 pixels, from other longitudes and distances."""
    va, pa = ts.make_views([10.0, 95.0, 200.0], (9, 7), 3.0, lat=12.0, dist=20.0)
    vb, pb = ts.make_views([40.0, 150.0], (6, 11), 3.4, lat=-20.0, dist=35.0)
    return np.concatenate([va, vb]), np.concatenate([pa, pb])


def test_gains_scale_each_view_of_a_uniform_box(ora):
    """A uniform unit cube projects to each ray's chord through the box;
    with gains every view's pixels carry their instrument's gain."""
    views, npix = _two_instruments()
    n, lo, hi = ts.box(8, 1.0)
    gains = np.array([0.7, 0.7, 0.7, 2.5, 2.5])
    g = ts.Geometry(n, lo, hi, views, npix, gains=gains)
    img = ora.project(g, np.ones(g.cube_shape()))
    k = 0
    for v in range(5):
        ncol, nrow = (int(t) for t in npix[v])
        for r in range(nrow):
            for c in range(ncol):
                d = ora.pixel_direction(views[v], npix[v], c, r)
                assert img[k] == pytest.approx(gains[v] * _chord(lo, hi, views[v][0:3], d), rel=1e-12, abs=1e-13)
                k += 1
    assert k == g.nrays


def test_gains_adjoint(ora):
    views, npix = _two_instruments()
    n, lo, hi = ts.box(9, 1.2)
    g = ts.Geometry(n, lo, hi, views, npix, gains=np.array([1.3, 1.3, 1.3, -0.4, 0.0]))
    rng = np.random.default_rng(8)
    x, y = rng.normal(size=g.cube_shape()), rng.normal(size=g.nrays)
    lhs = float(ora.project(g, x) @ y)
    rhs = float(np.sum(x * ora.backproject(g, y)))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_normal_operator_against_dense_matrices(ora):
    """A = M (P^T G^2 P + lam R D^T D R) M assembled from the dense Siddon
    rows, the per-ray gains, an explicit D and R, and a map mask."""
    views, npix = _two_instruments()
    n, lo, hi = ts.box(4, 1.3)
    rng = np.random.default_rng(9)
    mm = (rng.uniform(size=(4, 4, 4)) > 0.2).astype(np.uint8)
    gains = np.array([1.5, 1.5, 1.5, 0.6, 0.6])
    g = ts.Geometry(n, lo, hi, views, npix, map_mask=mm, gains=gains)
    height = (0.2, -0.1, 0.3, 0.5)
    lam = 0.37
    P = ora.dense_matrix(g)
    G = np.diag(np.repeat(gains, npix[:, 0] * npix[:, 1]))
    D = np.zeros((len(_pairs(n)), 64))
    for r, (a, b) in enumerate(_pairs(n)):
        D[r, a], D[r, b] = -1.0, 1.0
    R = np.diag(_heights_by_loops(g, height[:3], height[3]))
    M = np.diag(mm.reshape(-1).astype(float))
    A = M @ (P.T @ G @ G @ P + lam * R @ D.T @ D @ R) @ M
    x = rng.normal(size=64)
    got = ora.normal_operator(g, lam, height=height)(x.reshape(4, 4, 4)).reshape(-1)
    np.testing.assert_allclose(got, A @ x, rtol=1e-11, atol=1e-12)
    y = rng.normal(size=g.nrays)
    np.testing.assert_allclose(ora.rhs(g, y).reshape(-1), M @ P.T @ G @ y, rtol=1e-11, atol=1e-12)


def test_normal_operator_is_gradient_of_weighted_criterion(ora):
    """grad J = 2 (A x - b) for J = ||y - G P M x||^2 + lam ||D R M x||^2,
    J evaluated with np.diff on R M x (central differences)."""
    views, npix = _two_instruments()
    n, lo, hi = ts.box(5, 1.1)
    g = ts.Geometry(n, lo, hi, views, npix, gains=np.array([0.8, 0.8, 0.8, 1.9, 1.9]))
    height = (0.0, 0.0, 0.0, -0.2)
    rng = np.random.default_rng(10)
    x, y = rng.normal(size=g.cube_shape()), rng.normal(size=g.nrays)
    grad = 2.0 * (ora.normal_operator(g, 0.3, height=height)(x) - ora.rhs(g, y))
    for j in (0, 31, 62, 124):
        e = np.zeros(g.cube_shape())
        e.reshape(-1)[j] = 1.0
        hs = 1e-4
        fd = (ora.criterion(g, x + hs * e, y, 0.3, height=height)
              - ora.criterion(g, x - hs * e, y, 0.3, height=height)) / (2 * hs)
        assert fd == pytest.approx(float(grad.reshape(-1)[j]), rel=1e-6, abs=1e-6)


def test_two_instruments_recover_the_map(ora):
    """Noise-free data of two instruments with gains 0.6 and 2.2 on a 3^3
    cube seen by 5 views: the stacked operator has full column rank, so the
    unregularised least-squares solution with the gains is the map itself,
    and the same data read with unit gains give a different map."""
    views, npix = _two_instruments()
    n, lo, hi = ts.box(3, 1.0)
    gains = np.array([0.6, 0.6, 0.6, 2.2, 2.2])
    g = ts.Geometry(n, lo, hi, views, npix, gains=gains)
    e = np.random.default_rng(11).uniform(0.5, 2.0, size=g.cube_shape())
    y = ora.project(g, e)
    A = np.stack([ora.normal_operator(g, 0.0)(u.reshape(g.cube_shape())).reshape(-1)
                  for u in np.eye(27)], axis=1)
    assert np.linalg.cond(A) < 1e8
    sol = np.linalg.solve(A, ora.rhs(g, y).reshape(-1))
    np.testing.assert_allclose(sol, e.reshape(-1), rtol=1e-8)
    g1 = ts.Geometry(n, lo, hi, views, npix)
    A1 = np.stack([ora.normal_operator(g1, 0.0)(u.reshape(g.cube_shape())).reshape(-1)
                   for u in np.eye(27)], axis=1)
    sol1 = np.linalg.solve(A1, ora.rhs(g1, y).reshape(-1))
    assert np.abs(sol1 - e.reshape(-1)).max() > 0.1
