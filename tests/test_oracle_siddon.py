"""Pins for the oracle's line-of-sight projector (Eq. lo) and its transpose.

Nothing here compares the oracle with itself: each check is a hand-derived
fixture, a closed-form chord, a brute-force recomputation from the plain
definition (per-voxel slab clip), an exact matrix identity, or a symmetry of
the cube.
"""
import json
import os

import numpy as np
import pytest

import tomo_synth as ts

HERE = os.path.dirname(os.path.abspath(__file__))


def _dense_from_trace(ora, n, lo, hi, o, d):
    row = np.zeros(int(np.prod(n)))
    idx, ln, _ = ora.trace_ray(n, lo, hi, o, d)
    np.add.at(row, idx, ln)
    return row, idx, ln


# ---------------------------------------------------------------- golden


def test_hand_derived_segments(ora):
    """Segment lists derived on paper for a 4^3 unit-voxel box (ties, entry on
    a plane, rays lying in a plane, observer inside, misses)."""
    with open(os.path.join(HERE, "golden", "siddon_hand.json")) as f:
        gold = json.load(f)
    bx = gold["box"]
    for ray in gold["rays"]:
        idx, ln, tl = ora.trace_ray(bx["n"], bx["lo"], bx["hi"], ray["o"], ray["d"])
        dn = np.linalg.norm(ray["d"])
        assert idx.tolist() == ray["idx"], ray["name"]
        np.testing.assert_allclose(ln, np.array(ray["len_over_norm_d"]) * dn, rtol=1e-15,
                                   err_msg=ray["name"])
        assert tl.tolist() == ray["t_enter"], ray["name"]


# ---------------------------------------------------------- closed forms


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_axis_aligned_rays(ora, axis, sign):
    """A ray along an axis through voxel interiors crosses N voxels, each for
    exactly one voxel side, with consecutive indices."""
    n, lo, hi = (16, 16, 16), np.full(3, -1.5), np.full(3, 1.5)
    o = np.array([0.37, -0.81, 0.55])
    o[axis] = -215.0 * sign
    d = np.zeros(3)
    d[axis] = sign
    idx, ln, _ = ora.trace_ray(n, lo, hi, o, d)
    assert len(idx) == 16
    np.testing.assert_allclose(ln, 3.0 / 16, rtol=1e-12)
    step = int(sign) * [1, 16, 256][axis]
    assert np.all(np.diff(idx) == step)


@pytest.mark.parametrize(
    "o,d,chord",
    [
        ((-215.0, 0.3, -0.2), (2.0, 0.0, 0.0), 3.0),  # axis: L
        ((-215.0, -215.0, 0.01), (1.0, 1.0, 0.0), 3.0 * np.sqrt(2.0)),  # in-plane 45 deg: L sqrt 2
        ((-10.0, -10.0, -10.0), (1.0, 1.0, 1.0), 3.0 * np.sqrt(3.0)),  # space diagonal: L sqrt 3
        ((9.0, -9.0, 9.0), (-0.5, 0.5, -0.5), 3.0 * np.sqrt(3.0)),  # other diagonal, |d| != 1
    ],
)
def test_constant_cube_chords(ora, o, d, chord):
    """On a constant cube c the line integral is c times the chord; the
    chords along an axis, a face diagonal and the space diagonal of a box of
    side L are L, L sqrt 2 and L sqrt 3 (the last two pass through edges and
    corners, so every crossing is a tie)."""
    n, lo, hi = (12, 12, 12), np.full(3, -1.5), np.full(3, 1.5)
    idx, ln, _ = ora.trace_ray(n, lo, hi, o, d)
    assert abs(ln.sum() - chord) <= 1e-12 * chord
    c = 2.5
    assert abs(c * ln.sum() - c * chord) <= 1e-12 * c * chord
    # every segment positive (ties merged)
    assert np.all(ln > 0)


def test_space_diagonal_voxel_sequence(ora):
    """Through the corners every step advances all three axes at once: the
    sequence is the N diagonal voxels, each of length Delta sqrt 3."""
    n, lo, hi = (8, 8, 8), np.full(3, -1.0), np.full(3, 1.0)
    idx, ln, _ = ora.trace_ray(n, lo, hi, (-3.0, -3.0, -3.0), (1.0, 1.0, 1.0))
    assert idx.tolist() == [k * (64 + 8 + 1) for k in range(8)]
    np.testing.assert_allclose(ln, 0.25 * np.sqrt(3.0), rtol=1e-15)


def test_constant_cube_projection_equals_clip_length(ora):
    """P applied to a constant cube equals the constant times the chord of
    the box, for every pixel of a small pinhole geometry."""
    wl = ts.tiny()
    g = wl.geom
    c = 1.75
    img = ora.project(g, np.full(g.cube_shape(), c))
    # chord from the slab method, evaluated independently here
    chords = []
    for v in range(g.nviews):
        row = g.views[v]
        o = row[0:3]
        ncol, nrow = g.npix[v]
        for r in range(ncol * nrow):
            x = (r % ncol - row[14]) * row[12]
            y = (r // ncol - row[15]) * row[13]
            d = row[3:6] + x * row[6:9] + y * row[9:12]
            with np.errstate(divide="ignore"):
                t1, t2 = (g.lo - o) / d, (g.hi - o) / d
            tin = max(0.0, np.max(np.minimum(t1, t2)))
            tout = np.min(np.maximum(t1, t2))
            chords.append(max(0.0, tout - tin) * np.linalg.norm(d))
    chords = np.array(chords)
    np.testing.assert_allclose(img, c * chords, rtol=1e-12, atol=1e-14)
    assert np.count_nonzero(chords) > 0.5 * chords.size


# ------------------------------------------------------ vs brute force


def _random_rays(rng, n, lo, hi, count):
    rays = []
    span = hi - lo
    for _ in range(count):
        kind = rng.integers(0, 4)
        centre = lo + rng.uniform(-0.2, 1.2, 3) * span
        if kind == 0:  # general direction from outside
            d = rng.normal(size=3)
            o = centre - 3.0 * np.max(span) * d / np.linalg.norm(d)
        elif kind == 1:  # one zero direction component (parallel to a plane)
            d = rng.normal(size=3)
            d[rng.integers(0, 3)] = 0.0
            o = centre - 3.0 * np.max(span) * d / np.linalg.norm(d)
        elif kind == 2:  # two zero components (axis-parallel)
            d = np.zeros(3)
            d[rng.integers(0, 3)] = rng.choice([-1.0, 1.0]) * rng.uniform(0.5, 2)
            o = centre - 3.0 * np.max(span) * d / np.linalg.norm(d)
        else:  # origin inside the box
            o = lo + rng.uniform(0.05, 0.95, 3) * span
            d = rng.normal(size=3)
        rays.append((o, d))
    return rays


@pytest.mark.parametrize("n", [(4, 4, 4), (5, 7, 4), (16, 9, 11)])
def test_siddon_equals_per_voxel_slab(ora, n):
    """Each Siddon row equals the row computed voxel by voxel from the plain
    definition (length of the half-line inside each voxel box)."""
    rng = np.random.default_rng(sum(n))
    lo = rng.uniform(-2, -0.5, 3)
    hi = lo + rng.uniform(1.0, 3.0, 3)
    for o, d in _random_rays(rng, n, lo, hi, 60):
        row, idx, ln = _dense_from_trace(ora, n, lo, hi, o, d)
        bf = ora.ray_row_bruteforce(n, lo, hi, o, d)
        np.testing.assert_allclose(row, bf, atol=1e-12 * np.max(hi - lo), rtol=0)
        # each voxel is entered once: no repeated index, positive lengths
        assert len(np.unique(idx)) == len(idx)
        assert np.all(ln > 0)


DYADIC = [
    ((-3.0, 0.25, -0.375), (1.0, 0.25, 0.125)),
    ((0.5, -4.0, 0.125), (-0.25, 1.0, 0.5)),
    ((-3.0, -3.0, 0.0625), (1.0, 1.0, 0.0)),  # through lattice lines: ties
    ((2.0, 2.0, 3.0), (-0.5, -0.5, -1.0)),  # ties on two axes
    ((0.125, 0.375, -0.625), (0.75, -0.5, 0.25)),  # observer inside
    ((-5.0, 0.25, 0.25), (1.0, 0.0, 0.0)),  # lying on lattice planes y, z
]


@pytest.mark.parametrize("o,d", DYADIC)
def test_dyadic_rays_bit_exact(ora, o, d):
    """Box [-1, 1]^3, N = 16, dyadic origin and direction: every crossing
    parameter is exact, so the lengths equal the per-voxel slab lengths bit
    for bit and consecutive voxels differ by one step on each crossed axis."""
    n, lo, hi = (16, 16, 16), np.full(3, -1.0), np.full(3, 1.0)
    row, idx, ln = _dense_from_trace(ora, n, lo, hi, np.array(o), np.array(d))
    bf = ora.ray_row_bruteforce(n, lo, hi, np.array(o), np.array(d))
    assert np.array_equal(row, bf)
    ijk = np.stack([idx % 16, (idx // 16) % 16, idx // 256], axis=1)
    steps = np.diff(ijk, axis=0)
    sgn = np.sign(d).astype(int)
    for s in steps:
        for a in range(3):
            assert s[a] in (0, sgn[a])
        assert np.any(s != 0)


def test_shift_by_one_voxel_shifts_indices(ora):
    """Translating the ray by exactly one voxel side along x moves every
    interior segment to the neighbouring voxel with the same length."""
    n, lo, hi = (16, 16, 16), np.full(3, -1.0), np.full(3, 1.0)
    o, d = np.array([0.0, -3.0, 0.0625]), np.array([0.25, 1.0, 0.125])
    idx0, ln0, _ = ora.trace_ray(n, lo, hi, o, d)
    idx1, ln1, _ = ora.trace_ray(n, lo, hi, o + [0.125, 0, 0], d)
    common = [(i, l) for i, l in zip(idx0, ln0) if i % 16 < 15]
    shifted = dict(zip(idx1.tolist(), ln1.tolist()))
    for i, l in common:
        if i + 1 in shifted:
            assert shifted[i + 1] == l


# ------------------------------------------------------------ adjoint


def _tiny_geometry(npix=3, nviews=2, n=4):
    lons = [30.0 + 110.0 * k for k in range(nviews)]
    views, pix = ts.make_views(lons, (npix, npix), 3.2)
    nn, lo, hi = ts.box(n, 1.5)
    return ts.Geometry(nn, lo, hi, views, pix)


def test_transpose_matrix_is_exact(ora):
    """Columns of P (images of one-hot voxels) and rows of P (back-projections
    of one-hot pixels) give the same matrix, bit for bit."""
    g = _tiny_geometry()
    P = np.stack([ora.project(g, np.eye(g.nvox)[v].reshape(g.cube_shape()), 1)
                  for v in range(g.nvox)], axis=1)
    PT = np.stack([ora.backproject(g, np.eye(g.nrays)[r], 1).ravel()
                   for r in range(g.nrays)], axis=0)
    assert np.array_equal(P, PT)
    assert np.count_nonzero(P) > 0
    # and the dense matrix built ray by ray from traces agrees
    assert np.array_equal(P, ora.dense_matrix(g))


def test_adjoint_identity(ora):
    """<P x, y> = <x, P^T y> to rounding on random x, y."""
    wl = ts.tiny()
    g = wl.geom
    for seed in range(3):
        x, y = ts.random_pair(g.nvox, g.nrays, 500 + seed)
        lhs = float(ora.project(g, x.reshape(g.cube_shape())) @ y)
        rhs = float(x @ ora.backproject(g, y).ravel())
        assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(ora.project(g, x.reshape(g.cube_shape()))) * np.linalg.norm(y)


def test_backprojected_ones_sum_to_chords(ora):
    """sum_v (P^T 1)_v = sum over rays of the chord = sum of P 1."""
    g = ts.tiny().geom
    bp = ora.backproject(g, np.ones(g.nrays))
    chords = ora.project(g, np.ones(g.cube_shape()))
    assert abs(bp.sum() - chords.sum()) <= 1e-11 * chords.sum()


def test_one_hot_pixel_backprojects_its_segments(ora):
    g = ts.tiny().geom
    r = 5 * 32 + 17  # view 0, row 5, col 17
    bp = ora.backproject(g, np.eye(g.nrays)[r], 1).ravel()
    d = ora.pixel_direction(g.views[0], g.npix[0], 17, 5)
    row, _, _ = _dense_from_trace(ora, g.n, g.lo, g.hi, g.views[0][0:3], d)
    assert np.array_equal(bp, row)


# ---------------------------------------------------------- symmetries


def _rot_views(views, R):
    out = views.copy()
    for k in range(4):
        out[:, 3 * k:3 * k + 3] = views[:, 3 * k:3 * k + 3] @ R.T
    return out


def test_quarter_turn_symmetry(ora):
    """Turning observers and scene by 90 deg about z leaves every image
    unchanged (the symmetric box maps onto itself voxel for voxel)."""
    wl = ts.tiny()
    g = wl.geom
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])  # (x,y)->(-y,x)
    x = wl.x  # (z, y, x)
    N = x.shape[1]
    xr = np.empty_like(x)
    # voxel (i, j) with centre (c_i, c_j) moves to (-c_j, c_i) = (c_{N-1-j}, c_i)
    for j in range(N):
        for i in range(N):
            xr[:, i, N - 1 - j] = x[:, j, i]
    gr = ts.Geometry(g.n, g.lo, g.hi, _rot_views(g.views, R), g.npix)
    a = ora.project(g, x)
    b = ora.project(gr, xr)
    np.testing.assert_allclose(b, a, rtol=1e-11, atol=1e-12 * np.abs(a).max())


def test_mirror_symmetry(ora):
    wl = ts.tiny()
    g = wl.geom
    M = np.diag([1.0, -1.0, 1.0])
    xm = wl.x[:, ::-1, :].copy()
    gm = ts.Geometry(g.n, g.lo, g.hi, _rot_views(g.views, M), g.npix)
    a = ora.project(g, wl.x)
    b = ora.project(gm, xm)
    np.testing.assert_allclose(b, a, rtol=1e-11, atol=1e-12 * np.abs(a).max())


# --------------------------------------------------------------- physics


def test_gaussian_blob_line_integral(ora):
    """Sanity: the line integral of a Gaussian blob at impact parameter b is
    a sigma sqrt(2 pi) exp(-b^2 / 2 sigma^2).  An x-parallel ray crosses one
    column of voxels, so the voxelised sum is the midpoint rule along the line
    through that column's centres: it agrees with the closed form at the
    column's impact parameter to O((Delta/sigma)^2)."""
    n, lo, hi = ts.box(64, 1.5)
    delta = 3.0 / 64
    sig, amp = 0.3, 0.8
    x = ts.blob_cube(n, lo, hi, [(0.0, 0.0, 0.0, sig, amp)])
    for b in (0.0, 0.15, 0.3, 0.5):
        o, d = np.array([-215.0, b, 0.013]), np.array([1.0, 0.0, 0.0])
        idx, ln, _ = ora.trace_ray(n, lo, hi, o, d)
        val = float(np.sum(ln * x.ravel()[idx]))
        cy = -1.5 + (np.floor((b + 1.5) / delta) + 0.5) * delta
        cz = -1.5 + (np.floor((0.013 + 1.5) / delta) + 0.5) * delta
        bb = np.hypot(cy, cz)
        exact = amp * sig * np.sqrt(2 * np.pi) * np.exp(-bb * bb / (2 * sig * sig))
        assert abs(val - exact) <= 0.5 * (delta / sig) ** 2 * exact


# ---------------------------------------------------------------- masks


def test_data_and_map_masks(ora):
    wl = ts.tiny()
    g = wl.geom
    rng = np.random.default_rng(7)
    dm = (rng.uniform(size=g.nrays) > 0.3).astype(np.uint8)
    mm = (rng.uniform(size=g.cube_shape()) > 0.2).astype(np.uint8)
    gm = ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, data_mask=dm, map_mask=mm)
    full = ora.project(g, wl.x * mm)
    masked = ora.project(gm, wl.x)
    np.testing.assert_array_equal(masked[dm == 0], 0.0)
    np.testing.assert_allclose(masked[dm == 1], full[dm == 1], rtol=1e-14, atol=0)
    y = rng.normal(size=g.nrays)
    bp_full = ora.backproject(g, y * dm)
    bp = ora.backproject(gm, y)
    np.testing.assert_allclose(bp, bp_full * mm, rtol=1e-12, atol=1e-14)


def test_frames_select_their_cube(ora):
    wl = ts.tiny()
    g = wl.geom
    vf = np.arange(g.nviews, dtype=np.int32) % 3
    gf = ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, vf, 3)
    frames = np.stack([wl.x * (f + 1) for f in range(3)])
    img = ora.project(gf, frames)
    off = g.view_offsets()
    ref = ora.project(g, wl.x)
    for v in range(g.nviews):
        np.testing.assert_allclose(img[off[v]:off[v + 1]], (vf[v] + 1) * ref[off[v]:off[v + 1]],
                                   rtol=1e-14)
    y = np.random.default_rng(3).normal(size=g.nrays)
    bp = ora.backproject(gf, y)
    for f in range(3):
        sel = np.zeros(g.nrays)
        for v in np.nonzero(vf == f)[0]:
            sel[off[v]:off[v + 1]] = 1.0
        np.testing.assert_allclose(bp[f], ora.backproject(g, y * sel), rtol=1e-12, atol=1e-14)


def test_crossing_count_equals_nonzero_entries(ora):
    g = _tiny_geometry(npix=6, nviews=3, n=5)
    P = ora.dense_matrix(g)
    assert ora.count_crossings(g) == np.count_nonzero(P)
    dm = np.zeros(g.nrays, dtype=np.uint8)
    dm[::2] = 1
    gm = ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, data_mask=dm)
    assert ora.count_crossings(gm) == np.count_nonzero(P[::2])
