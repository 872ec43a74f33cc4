"""Pins of the oracle's Thomson-scattering operators (Sec. "White Light:
Thomson Scattering"; Eq. 4C, Eq. thomson_lo, Eq. brightness and
Eq. thomson_direct): Billings' coefficients at a hand-computed angle, their
small-angle limits (a point source; the 2/3 flux of a linearly
limb-darkened disc), their values at the limb, B >= pB, the impact
parameter in closed form, the operators on single voxels, and adjointness."""
import numpy as np
import pytest

import tomo_synth as ts


def test_coefficients_at_30_degrees(ora):
    """sin(Omega) = 1/2, cos(Omega) = sqrt(3)/2, ln((1 + s)/c) = ln(3)/2."""
    c1, c2, c3, c4 = ora.thomson_c1234(np.array([0.5]))
    l3 = np.log(3.0)
    assert c1[0] == pytest.approx(np.sqrt(3.0) / 8.0, rel=1e-14)
    assert c2[0] == pytest.approx(-1.0 / 32.0 + 21.0 / 128.0 * l3, rel=1e-14)
    assert c3[0] == pytest.approx(4.0 / 3.0 - 5.0 * np.sqrt(3.0) / 8.0, rel=1e-14)
    assert c4[0] == pytest.approx(21.0 / 32.0 - 57.0 / 128.0 * l3, rel=1e-14)


def test_small_angle_limits(ora):
    """Far from the Sun the disc is a point source of solid angle ~ pi s^2:
    C1 and C3 tend to s^2, and the limb-darkened coefficients C2 and C4 to
    2/3 of them (a disc of brightness 1 - u + u cos(psi) radiates 1 - u/3 of
    its u = 0 flux)."""
    s = np.array([1e-2])
    c1, c2, c3, c4 = ora.thomson_c1234(s)
    assert c1[0] / s[0] ** 2 == pytest.approx(1.0, abs=1e-3)
    assert c3[0] / s[0] ** 2 == pytest.approx(1.0, abs=1e-3)
    assert c2[0] / c1[0] == pytest.approx(2.0 / 3.0, abs=1e-3)
    assert c4[0] / c3[0] == pytest.approx(2.0 / 3.0, abs=1e-3)


def test_limb_values(ora):
    """At the limb (s -> 1, cos -> 0; cos^2 ln(1/cos) -> 0): C1 -> 0,
    C2 -> 1/4, C3 -> 4/3, C4 -> 3/4."""
    c1, c2, c3, c4 = ora.thomson_c1234(np.array([1.0 - 1e-12]))
    assert c1[0] == pytest.approx(0.0, abs=1e-5)
    assert c2[0] == pytest.approx(0.25, abs=1e-4)
    assert c3[0] == pytest.approx(4.0 / 3.0, abs=1e-5)
    assert c4[0] == pytest.approx(0.75, abs=1e-4)


def test_total_exceeds_polarized_brightness(ora):
    """In the plane of the sky (rho = r) B - pB = 2 I_r >= 0, i.e. the
    C3/C4 combination is at least the C1/C2 one, and both are positive."""
    s = np.linspace(0.01, 0.999, 400)
    c1, c2, c3, c4 = ora.thomson_c1234(s)
    for u in (0.0, 0.3, 0.6, 1.0):
        a = (1 - u) * c1 + u * c2
        b = (1 - u) * c3 + u * c4
        assert np.all(a > 0) and np.all(b >= a)


def test_impact_parameter_closed_form(ora):
    """An observer at distance D aimed at the Sun's centre: a pixel at
    tangent-plane offset x from the reference has rho^2 = D^2 x^2 / (1 + x^2);
    the reference pixel's line passes through the centre (rho = 0)."""
    views, npix = ts.make_views([30.0], (5, 3), 3.0, dist=20.0)
    g = ts.Geometry((4, 4, 4), np.full(3, -1.0), np.full(3, 1.0), views, npix)
    o = ora.thomson_pixel_weights(g)
    cd = views[0, 12]
    for row in range(3):
        for col in range(5):
            x2 = ((col - 2) * cd) ** 2 + ((row - 1) * cd) ** 2
            assert o[row * 5 + col] == pytest.approx(400.0 * x2 / (1.0 + x2), rel=1e-12, abs=1e-24)


def _geom():
    n, lo, hi = ts.box(10, 2.5)
    views, npix = ts.make_views([0.0, 70.0, 150.0, 230.0], (12, 10), 6.0, lat=10.0, dist=30.0)
    return ts.Geometry(n, lo, hi, views, npix)


@pytest.mark.parametrize("kind", ["pB", "B"])
def test_single_voxel_columns(ora, kind):
    """The column of voxel j: pB_k = scale rho_k^2 m_j l_kj and
    B_k = scale (m'_j - rho_k^2 m_j) l_kj, l_kj from the Siddon trace."""
    g = _geom()
    u, scale = 0.6, 2.5
    m, mp = ora.thomson_voxel_weights(g, u)
    o = ora.thomson_pixel_weights(g)
    j = (7 * 10 + 2) * 10 + 5  # a voxel outside the photosphere
    assert m.reshape(-1)[j] > 0
    e = np.zeros(g.cube_shape())
    e.reshape(-1)[j] = 1.0
    col = ora.thomson_project(g, e, u, kind, scale)
    ell = ora.project(g, e)
    w = o * m.reshape(-1)[j] if kind == "pB" else mp.reshape(-1)[j] - o * m.reshape(-1)[j]
    np.testing.assert_allclose(col, scale * w * ell, rtol=1e-13, atol=1e-300)
    assert np.count_nonzero(ell) > 0


def test_weights_vanish_inside_the_photosphere(ora):
    g = _geom()
    m, mp = ora.thomson_voxel_weights(g, 0.5)
    nx = g.n[0]
    cen = g.lo[0] + (np.arange(nx) + 0.5) * (g.hi[0] - g.lo[0]) / nx
    zz, yy, xx = np.meshgrid(cen, cen, cen, indexing="ij")
    inside = xx ** 2 + yy ** 2 + zz ** 2 <= 1.0
    assert np.all(m[inside] == 0) and np.all(mp[inside] == 0)
    assert np.all(m[~inside] > 0) and np.all(mp[~inside] > m[~inside])


@pytest.mark.parametrize("kind", ["pB", "B"])
def test_adjoint(ora, kind):
    g = _geom()
    rng = np.random.default_rng(7)
    x, y = rng.normal(size=g.cube_shape()), rng.normal(size=g.nrays)
    lhs = float(np.dot(ora.thomson_project(g, x, 0.55, kind, 1.7), y))
    rhs = float(np.sum(x * ora.thomson_backproject(g, y, 0.55, kind, 1.7)))
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("u", [0.0, 0.4, 1.0])
def test_weights_point_source_limit(ora, u):
    """Far away (r = 200 R_sun) the Sun is a point source whose limb-darkened
    flux is 1 - u/3 of the uniform disc's: m r^6 -> 1 - u/3 and
    m' r^4 / 2 -> 1 - u/3, the weights' u combination and powers of r checked
    against the physical limit rather than their formulas."""
    views, npix = ts.make_views([0.0], (2, 2), 1.0, dist=400.0)
    g = ts.Geometry((1, 1, 1), np.array([199.5, -0.5, -0.5]), np.array([200.5, 0.5, 0.5]), views, npix)
    m, mp = ora.thomson_voxel_weights(g, u)
    r = 200.0
    assert float(m.reshape(-1)[0]) * r ** 6 == pytest.approx(1.0 - u / 3.0, rel=1e-4)
    assert float(mp.reshape(-1)[0]) * r ** 4 / 2.0 == pytest.approx(1.0 - u / 3.0, rel=1e-4)
