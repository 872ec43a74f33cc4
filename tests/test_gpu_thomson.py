"""GPU parity of the Thomson-scattering operators (Sec. "White Light:
Thomson Scattering", Eq. thomson_direct) against the FP64 oracle, through the
C ABI: pB = scale O P M n_e and B = scale (P M' - O P M) n_e, and their
transposes, on a coronagraph-like geometry (box [-4, 4]^3 R_sun, detector
annulus 1.4-4 R_sun kept, the unit sphere masked)."""
import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import assert_p_close, length_resolution, need_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

U, SCALE = 0.63, 3.0


@pytest.fixture(scope="module")
def tomo():
    return need_gpu()


def _cor1_like(n=40, npix=64, nviews=6):
    nn, lo, hi = ts.box(n, 4.0)
    views, pix = ts.make_views(np.linspace(0.0, 300.0, nviews), (npix, npix), 8.0, lat=7.0)
    dm = ts.annulus_data_mask(views, pix, 1.4, 4.0)
    mm = ts.sphere_map_mask(nn, lo, hi, 1.0)
    return ts.Geometry(nn, lo, hi, views, pix, data_mask=dm, map_mask=mm)


def _abs_refs(ora, g, x, y, kind):
    """Oracle values and the magnitudes the error bounds scale with: the
    operator with every term counted positive, on |x| and |y|."""
    m, mp = ora.thomson_voxel_weights(g, U)
    o = ora.thomson_pixel_weights(g)
    ax, ay = np.abs(x), np.abs(y)
    if kind == "pB":
        fa = SCALE * o * ora.project(g, ax * m)
        ba = SCALE * m * ora.backproject(g, o * ay)
    else:
        fa = SCALE * (ora.project(g, ax * mp) + o * ora.project(g, ax * m))
        ba = SCALE * (mp * ora.backproject(g, ay) + m * ora.backproject(g, o * ay))
    return (ora.thomson_project(g, x, U, kind, SCALE), fa,
            ora.thomson_backproject(g, y, U, kind, SCALE), ba)


@pytest.mark.parametrize("kind", ["pB", "B"])
def test_every_pixel_and_voxel(tomo, ora, kind):
    g = _cor1_like()
    rng = np.random.default_rng(50)
    x = rng.uniform(size=g.cube_shape())
    y = rng.normal(size=g.nrays)
    fv, fa, bv, ba = _abs_refs(ora, g, x, y, kind)
    dg = tomo.DeviceGeometry(g)
    res = length_resolution(g)
    got = to_host(tomo.thomson_project(dg, to_dev(x), U, kind, SCALE))
    assert_p_close(got, fv, fa, what=f"T_{kind}", atol=res * float(np.max(np.abs(fa))))
    assert np.count_nonzero(got) > 0.3 * g.nrays
    gotb = to_host(tomo.thomson_backproject(dg, to_dev(y), U, kind, SCALE))
    assert_p_close(gotb, bv, ba, rtol=1e-4, what=f"T_{kind}^T", atol=res * float(np.max(np.abs(ba))))


@pytest.mark.parametrize("kind", ["pB", "B"])
def test_accumulate_and_adjoint(tomo, kind):
    g = _cor1_like(n=24, npix=48, nviews=4)
    dg = tomo.DeviceGeometry(g)
    rng = np.random.default_rng(51)
    x, y = rng.normal(size=g.cube_shape()), rng.normal(size=g.nrays)
    tx = to_host(tomo.thomson_project(dg, to_dev(x), U, kind, SCALE))
    tty = tomo.thomson_backproject(dg, to_dev(y), U, kind, SCALE)
    lhs, rhs = float(np.dot(tx, y)), float(np.sum(x * to_host(tty)))
    scale = float(np.dot(np.abs(tx), np.abs(y))) + 1e-30
    assert abs(lhs - rhs) <= 1e-5 * scale
    base = to_dev(rng.normal(size=g.cube_shape()))
    acc = base.clone()
    tomo.thomson_backproject(dg, to_dev(y), U, kind, SCALE, out=acc, accumulate=True)
    np.testing.assert_allclose(to_host(acc), to_host(base) + to_host(tty), rtol=1e-6, atol=1e-6)


def test_sun_off_centre_and_units(tomo, ora):
    """The Sun's centre off the box centre and the box in units of 2 R_sun:
    the same operator as the oracle's with sun = (cx, cy, cz, R)."""
    g = _cor1_like(n=24, npix=48, nviews=4)
    sun = (0.3, -0.2, 0.1, 0.5)
    dg = tomo.DeviceGeometry(g)
    rng = np.random.default_rng(52)
    x = rng.uniform(size=g.cube_shape())
    ref = ora.thomson_project(g, x, U, "B", SCALE, sun)
    m, mp = ora.thomson_voxel_weights(g, U, sun)
    o = ora.thomson_pixel_weights(g, sun)
    fa = SCALE * (ora.project(g, x * mp) + o * ora.project(g, x * m))
    got = to_host(tomo.thomson_project(dg, to_dev(x), U, "B", SCALE, sun))
    assert_p_close(got, ref, fa, what="T_B", atol=length_resolution(g) * float(np.max(fa)))
