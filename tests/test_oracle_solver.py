"""Pins for the oracle's priors and solvers (Eq. criterion, Eq. stsrt).

The finite-difference prior is pinned by the spectrum of a path-graph
Laplacian; CG by a dense direct solve, its closed-form first step and the
monotone criterion the paper plots; FCG by an exact identity network.
"""
import numpy as np
import pytest

import tomo_synth as ts


def _dense_op(f, shape):
    n = int(np.prod(shape))
    return np.stack([f(np.eye(n)[k].reshape(shape)).ravel() for k in range(n)], axis=1)


def test_laplacian6_structure(ora):
    shape = (3, 5, 4)  # (nz, ny, nx)
    L = _dense_op(ora.laplacian6, shape)
    assert np.array_equal(L, L.T)
    np.testing.assert_allclose(L @ np.ones(L.shape[0]), 0.0, atol=1e-14)
    # interior voxel (z=1, y=2, x=1): 6 on the diagonal, -1 on 6 neighbours
    c = (1 * 5 + 2) * 4 + 1
    nb = [c - 1, c + 1, c - 4, c + 4, c - 20, c + 20]
    assert L[c, c] == 6.0
    assert all(L[c, k] == -1.0 for k in nb)
    assert np.count_nonzero(L[c]) == 7
    # corner voxel: 3 in-cube neighbours
    assert L[0, 0] == 3.0


def test_laplacian6_spectrum(ora):
    """D^T D of a box grid is the Cartesian sum of path-graph Laplacians, whose
    eigenvalues are 2 - 2 cos(pi k / N), k = 0..N-1."""
    shape = (3, 4, 5)
    L = _dense_op(ora.laplacian6, shape)
    ev = np.sort(np.linalg.eigvalsh(L))
    path = [2 - 2 * np.cos(np.pi * np.arange(m) / m) for m in shape]
    expect = np.sort((path[0][:, None, None] + path[1][None, :, None] + path[2][None, None, :]).ravel())
    np.testing.assert_allclose(ev, expect, atol=1e-12)


def test_laplacian_t(ora):
    shape = (4, 2, 2, 3)
    L = _dense_op(ora.laplacian_t, shape)
    assert np.array_equal(L, L.T)
    ev = np.sort(np.linalg.eigvalsh(L))
    path = 2 - 2 * np.cos(np.pi * np.arange(4) / 4)
    np.testing.assert_allclose(ev, np.sort(np.repeat(path, 12)), atol=1e-12)
    x = np.random.default_rng(0).normal(size=shape)
    lt = ora.laplacian_t(x)
    np.testing.assert_allclose(lt[1], 2 * x[1] - x[0] - x[2], atol=1e-14)
    np.testing.assert_allclose(lt[0], x[0] - x[1], atol=1e-14)
    np.testing.assert_allclose(lt[3], x[3] - x[2], atol=1e-14)


def _small_problem(ora, mask=False, frames=1):
    n = 4
    views, pix = ts.make_views([20.0, 80.0, 150.0, 260.0], (4, 4), 3.2)
    nn, lo, hi = ts.box(n, 1.5)
    vf = None if frames == 1 else (np.arange(4) % frames).astype(np.int32)
    mm = None
    if mask:
        mm = np.ones((n, n, n), dtype=np.uint8)
        mm[1:3, 1:3, 1:3] = 0
    g = ts.Geometry(nn, lo, hi, views, pix, vf, frames, map_mask=mm)
    rng = np.random.default_rng(11)
    x = rng.uniform(size=g.cube_shape())
    y = ora.project(g, x) + 0.01 * rng.normal(size=g.nrays)
    return g, y


@pytest.mark.parametrize("mask,frames,lam_t", [(False, 1, 0.0), (True, 1, 0.0), (False, 2, 10.0)])
def test_cg_matches_dense_solve(ora, mask, frames, lam_t):
    g, y = _small_problem(ora, mask, frames)
    lam = 1e-2
    A = ora.normal_operator(g, lam, lam_t)
    b = ora.rhs(g, y)
    shape = g.cube_shape()
    Ad = _dense_op(A, shape)
    bd = b.ravel()
    if mask:  # restrict to the kept voxels (the operator is P M)
        keep = np.tile(g.map_mask.ravel(), frames).astype(bool)
        xs = np.zeros(bd.size)
        xs[keep] = np.linalg.solve(Ad[np.ix_(keep, keep)], bd[keep])
    else:
        xs = np.linalg.solve(Ad, bd)
    x, hist = ora.cg(A, b, n_iter=400, rtol=1e-12)
    assert np.linalg.norm(x.ravel() - xs) <= 1e-8 * np.linalg.norm(xs)
    if mask:
        assert np.all(x.reshape(shape)[..., g.map_mask == 0] == 0)


def test_cg_first_step_closed_form(ora):
    """From x0 = 0 the first CG iterate is the exact line minimiser along b:
    x1 = (b.b / b.A b) b."""
    wl = ts.tiny()
    g = wl.geom
    A = ora.normal_operator(g, 1e-2)
    y = ora.project(g, wl.x)
    b = ora.rhs(g, y)
    x1, _ = ora.cg(A, b, n_iter=1)
    expect = float(np.vdot(b, b)) / float(np.vdot(b, A(b))) * b
    np.testing.assert_allclose(x1, expect, rtol=1e-12, atol=1e-15)


def test_cg_criterion_decreases(ora):
    """The criterion J (Eq. criterion) decreases at every CG iteration, as in
    the paper's convergence plot."""
    wl = ts.tiny()
    g = wl.geom
    y = ora.project(g, wl.x)
    A = ora.normal_operator(g, wl.lam_r)
    x, hist, its = ora.cg(A, ora.rhs(g, y), n_iter=20, record=True)
    J = [ora.criterion(g, xi, y, wl.lam_r) for xi in its]
    assert all(J[k + 1] < J[k] for k in range(len(J) - 1))
    assert hist[-1] < 0.1 * hist[0]


def test_normal_operator_is_gradient_of_criterion(ora):
    """grad J = 2 (A x - b): checked by central differences of J along a
    random direction (J is quadratic, so the difference quotient is exact up
    to rounding)."""
    wl = ts.tiny()
    g = wl.geom
    y = ora.project(g, wl.x)
    A = ora.normal_operator(g, 0.3)
    b = ora.rhs(g, y)
    rng = np.random.default_rng(5)
    x = rng.normal(size=g.cube_shape())
    e = rng.normal(size=g.cube_shape())
    h = 1e-3
    fd = (ora.criterion(g, x + h * e, y, 0.3) - ora.criterion(g, x - h * e, y, 0.3)) / (2 * h)
    an = 2.0 * float(np.vdot(A(x) - b, e))
    assert abs(fd - an) <= 1e-7 * abs(an)


@pytest.mark.parametrize("scale", [1.0, 3.5])
def test_fcg_with_identity_network_reproduces_cg(ora, scale):
    g, y = _small_problem(ora)
    A = ora.normal_operator(g, 1e-2)
    b = ora.rhs(g, y)
    net = ora.normalized_precond(ora.identity_net(scale))
    r = np.random.default_rng(0).normal(size=b.shape)
    np.testing.assert_allclose(net(r), scale * r, rtol=1e-13, atol=1e-15)
    _, h_cg = ora.cg(A, b, n_iter=15)
    _, h_fcg, fb = ora.fcg(A, b, net, n_iter=15)
    assert fb == -1
    np.testing.assert_allclose(h_fcg, h_cg, rtol=1e-6)


def _stalling_net(ora, c):
    """z = r + c (r_{x+1} - r_{x-1}): the skew part adds nothing to z.r, so
    z.r = r.r > 0, but for large c the step is almost orthogonal to r and the
    residual barely moves."""
    h = np.zeros((3, 3, 3))
    h[1, 1, 1] = 1.0
    h[1, 1, 2], h[1, 1, 0] = c, -c
    return ora.linear_filter_net(h)


def test_fcg_survives_a_poor_network(ora):
    """A network that adds a large skew term still converges under FCG (the
    Polak-Ribiere beta cancels a repeated bad component)."""
    g, y = _small_problem(ora)
    A = ora.normal_operator(g, 1e-2)
    b = ora.rhs(g, y)
    bad = ora.normalized_precond(_stalling_net(ora, 1e4))
    r = np.random.default_rng(1).normal(size=b.shape)
    assert abs(float(np.vdot(bad(r), r)) - float(np.vdot(r, r))) <= 1e-9 * float(np.vdot(r, r))
    x, hist, fb = ora.fcg(A, b, bad, n_iter=400, rtol=1e-6)
    assert hist[-1] <= 1e-6


def test_fcg_falls_back_after_three_stalls(ora):
    """A preconditioner that adds a fresh, huge random component orthogonal
    to r at every call keeps z.r = r.r > 0 but makes almost no progress: after
    three non-falling iterations the solver restarts as plain CG, which then
    converges like CG from scratch."""
    g, y = _small_problem(ora)
    A = ora.normal_operator(g, 1e-2)
    b = ora.rhs(g, y)
    rng = np.random.default_rng(42)

    def bad(r):
        q = rng.normal(size=r.shape)
        q -= float(np.vdot(q, r)) / float(np.vdot(r, r)) * r
        return r + 1e8 * np.linalg.norm(r) * q / np.linalg.norm(q)

    x, hist, fb = ora.fcg(A, b, bad, n_iter=400, rtol=1e-6)
    assert fb == 3
    assert all(hist[k + 1] > (1 - 1e-6) * hist[k] for k in range(3))
    assert hist[-1] <= 1e-6
    _, h_cg = ora.cg(A, b, n_iter=400, rtol=1e-6)
    assert abs((len(hist) - 4) - (len(h_cg) - 1)) <= 3


def test_fcg_skew_network_falls_back_at_once(ora):
    """A purely skew network gives z.r = 0 up to rounding: no descent
    direction, so the solver must not divide by it."""
    g, y = _small_problem(ora)
    A = ora.normal_operator(g, 1e-2)
    b = ora.rhs(g, y)
    h = np.zeros((3, 3, 3))
    h[1, 1, 2], h[1, 1, 0] = 1.0, -1.0
    skew = ora.normalized_precond(ora.linear_filter_net(h))
    x, hist, fb = ora.fcg(A, b, skew, n_iter=400, rtol=1e-6)
    assert fb in (0, 3)
    assert np.all(np.isfinite(hist)) and hist[-1] <= 1e-6
