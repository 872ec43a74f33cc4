"""Host-side checks of the C ABI (no GPU work is launched): the library loads,
exports every function the header declares, validates geometries, and its
WCS conversion agrees with the oracle's independent one."""
import ctypes
import os
import re

import numpy as np
import pytest

import tomo_synth as ts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def tomo():
    import paper_1103_5904_amd as t

    if not os.path.exists(t.tomo.LIB_PATH):
        from paper_1103_5904_amd import build

        build.build()
    return t


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(tomo_[a-z0-9_]+)\s*\(", txt))
    return names


def test_exports_every_declared_function(tomo):
    names = _declared()
    assert {"tomo_project", "tomo_backproject", "tomo_cg_solve"} <= names
    L = ctypes.CDLL(tomo.tomo.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    assert set(tomo.tomo.EXPORTS) <= names


def _geom(**over):
    wl = ts.tiny()
    g = wl.geom
    views = g.views.copy()
    npix = g.npix.copy()
    for k, v in over.items():
        if k == "views":
            views = v
        elif k == "npix":
            npix = v
    return ts.Geometry(over.get("n", g.n), over.get("lo", g.lo), over.get("hi", g.hi), views, npix,
                       over.get("view_frame"), over.get("nframes", 1))


def test_validation_accepts_the_tiny_geometry(tomo):
    dg = tomo.DeviceGeometry(_geom(), device="cpu")
    assert tomo.validate(dg) == 0
    assert tomo.lib().tomo_geometry_pixels(dg.ref) == 8 * 32 * 32


def test_validation_accepts_a_cube_of_2_30_voxels(tomo):
    dg = tomo.DeviceGeometry(_geom(n=(1024, 1024, 1024)), device="cpu")
    assert tomo.validate(dg) == 0


@pytest.mark.parametrize("case", ["zero_dim", "inverted_box", "non_unit_w", "non_orthogonal",
                                  "zero_cdelt", "empty_image", "bad_frame", "nan_obs", "huge_cube",
                                  "long_side"])
def test_validation_rejects(tomo, case):
    g = _geom()
    views, npix = g.views.copy(), g.npix.copy()
    kw = {}
    if case == "zero_dim":
        kw["n"] = (0, 32, 32)
    elif case == "inverted_box":
        kw["hi"] = np.array([1.5, -2.0, 1.5])
    elif case == "non_unit_w":
        views[0, 3:6] *= 1.01
    elif case == "non_orthogonal":
        views[1, 6:9] = views[1, 3:6]
    elif case == "zero_cdelt":
        views[2, 12] = 0.0
    elif case == "empty_image":
        npix[3, 0] = 0
    elif case == "bad_frame":
        kw["view_frame"] = np.full(g.nviews, 1, dtype=np.int32)
    elif case == "nan_obs":
        views[0, 0] = np.nan
    elif case == "huge_cube":  # one voxel plane above 2^30
        kw["n"] = (1024, 1024, 1025)
    elif case == "long_side":  # under 2^30 voxels, but a side above 2^24
        kw["n"] = (1, (1 << 24) + 1, 1)
    dg = tomo.DeviceGeometry(_geom(views=views, npix=npix, **kw), device="cpu")
    assert tomo.validate(dg) == tomo.tomo.TOMO_EINVAL
    assert tomo.lib().tomo_last_error()


def test_null_arguments_are_rejected_without_gpu_work(tomo):
    L = tomo.lib()
    dg = tomo.DeviceGeometry(_geom(), device="cpu")
    assert L.tomo_project(dg.ref, None, None, None) == tomo.tomo.TOMO_EINVAL
    assert L.tomo_backproject(dg.ref, None, None, 0, None) == tomo.tomo.TOMO_EINVAL
    assert L.tomo_project(None, None, None, None) == tomo.tomo.TOMO_EINVAL
    assert L.tomo_validate_geometry(None) == tomo.tomo.TOMO_EINVAL
    assert tomo.status_string(tomo.tomo.TOMO_ENONFINITE) == "non-finite value in the solver"


def test_tuning_round_trip_and_range_checks(tomo):
    old = tomo.get_tuning()
    try:
        assert old["bp_ray_table"] == 1  # the default: solves and batches set each ray up once
        tomo.set_tuning(p_bundle=4, bp_lds_bins=2048, bp_ray_table=0)
        t = tomo.get_tuning()
        assert t["p_bundle"] == 4 and t["bp_lds_bins"] == 2048 and t["bp_ray_table"] == 0
        for bad in ({"p_bundle": 5}, {"bp_lds_bins": 100}, {"bp_default": 7}, {"p_xcd_remap": 3},
                    {"bp_ray_table": 2}, {"bp_ray_table": -1}):
            with pytest.raises(tomo.TomoError):
                tomo.set_tuning(**bad)
        assert tomo.get_tuning() == t  # unchanged by rejected calls
    finally:
        tomo.set_tuning(**old)


@pytest.mark.parametrize("args", [
    (215.0, 0.0, 0.0, 0.0, 0.0, 0.0, 2.0, 2.0, 16.5, 16.5, 32, 32),
    (212.3, 73.0, 4.5, 950.0, -420.0, 12.0, 1.6, 1.7, 256.5, 250.0, 512, 500),
    (30.0, -140.0, -7.0, -3000.0, 2500.0, -95.0, 14.0, 14.0, 1.0, 64.0, 128, 128),
])
def test_wcs_matches_the_oracle(tomo, ora, args):
    row_lib, pix_lib = tomo.view_from_wcs(*args)
    row_ora, pix_ora = ora.view_from_wcs(*args)
    np.testing.assert_allclose(row_lib, row_ora, rtol=1e-12, atol=1e-12)
    assert list(pix_lib) == list(pix_ora)


def test_wcs_rejects_bad_keywords(tomo):
    with pytest.raises(tomo.TomoError):
        tomo.view_from_wcs(0.0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 8, 8)
    with pytest.raises(tomo.TomoError):
        tomo.view_from_wcs(215.0, np.nan, 0, 0, 0, 0, 1, 1, 1, 1, 8, 8)


@pytest.mark.parametrize("case", ["u_high", "u_nan", "radius", "kind", "centre"])
def test_thomson_parameters_rejected(tomo, case):
    """Invalid Thomson parameters return TOMO_EINVAL before any device work."""
    dg = tomo.DeviceGeometry(_geom(), device="cpu")
    u, scale, sun, kind = 0.6, 1.0, [0.0, 0.0, 0.0, 1.0], 0
    if case == "u_high":
        u = 1.5
    elif case == "u_nan":
        u = float("nan")
    elif case == "radius":
        sun[3] = 0.0
    elif case == "kind":
        kind = 2
    elif case == "centre":
        sun[1] = float("inf")
    t = tomo.tomo._thomson_params(u, scale, sun)
    rc = tomo.lib().tomo_thomson_project(dg.ref, ctypes.byref(t), kind, ctypes.c_void_p(16), ctypes.c_void_p(16),
                                         None)
    assert rc == tomo.tomo.TOMO_EINVAL
    assert tomo.lib().tomo_last_error()


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_gain_rejected(tomo, bad):
    g = _geom()
    gains = np.ones(g.nviews)
    gains[3] = bad
    dg = tomo.DeviceGeometry(ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, gains=gains), device="cpu")
    assert tomo.validate(dg) == tomo.tomo.TOMO_EINVAL
    assert b"gain" in tomo.lib().tomo_last_error()


def test_gains_accepted_and_checked_for_length(tomo):
    g = _geom()
    gains = np.linspace(0.5, 2.0, g.nviews)
    dg = tomo.DeviceGeometry(ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, gains=gains), device="cpu")
    assert tomo.validate(dg) == 0
    with pytest.raises(ValueError):
        tomo.DeviceGeometry(ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, gains=gains[:-1]), device="cpu")


@pytest.mark.parametrize("height", [(np.nan, 0.0, 0.0, 0.0), (0.0, 0.0, 0.0, np.inf)])
def test_height_parameters_rejected(tomo, height):
    """A non-finite height centre or offset returns TOMO_EINVAL before any
    device work."""
    dg = tomo.DeviceGeometry(_geom(), device="cpu")
    h = tomo.tomo._height(height)
    rc = tomo.lib().tomo_apply_height_prior(ctypes.byref(dg.g.cube), ctypes.byref(h), 1.0, 0.0,
                                            ctypes.c_void_p(16), ctypes.c_void_p(32), 0, None)
    assert rc == tomo.tomo.TOMO_EINVAL
    assert b"height" in tomo.lib().tomo_last_error()
