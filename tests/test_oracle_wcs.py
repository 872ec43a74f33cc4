"""Pins for the oracle's reading of helioprojective TAN WCS keywords."""
import numpy as np
import pytest

import tomo_synth as ts

A2R = np.pi / (180 * 3600)


def test_earth_facing_frame(ora):
    row, pix = ora.view_from_wcs(215.0, 0.0, 0.0, 0.0, 0.0, 0.0, 2.0, 2.0, 16.5, 16.5, 32, 32)
    np.testing.assert_allclose(row[0:3], [215.0, 0, 0], atol=1e-12)
    np.testing.assert_allclose(row[3:6], [-1.0, 0, 0], atol=1e-15)  # toward the Sun
    np.testing.assert_allclose(row[6:9], [0, 1.0, 0], atol=1e-15)  # west
    np.testing.assert_allclose(row[9:12], [0, 0, 1.0], atol=1e-15)  # north
    np.testing.assert_allclose(row[12:14], 2.0 * A2R, rtol=1e-15)
    np.testing.assert_allclose(row[14:16], 15.5)  # FITS 1-based -> 0-based


@pytest.mark.parametrize("lon,lat", [(0.0, 0.0), (73.0, 0.0), (-120.0, 7.25), (200.0, -5.0)])
def test_reference_pixel_points_at_crval(ora, lon, lat):
    tx_as, ty_as = 950.0, -420.0
    row, pix = ora.view_from_wcs(215.0, lon, lat, tx_as, ty_as, 0.0, 1.5, 1.5, 10.0, 12.0, 20, 24)
    obs, w, u, v = row[0:3], row[3:6], row[6:9], row[9:12]
    S = -obs / np.linalg.norm(obs)
    N = np.array([0, 0, 1.0]) - S[2] * S
    N /= np.linalg.norm(N)
    W = np.cross(S, N)
    d = ora.pixel_direction(row, pix, 9, 11)  # crpix - 1
    d = d / np.linalg.norm(d)
    tx = np.arctan2(d @ W, d @ S)
    ty = np.arcsin(d @ N)
    np.testing.assert_allclose([tx, ty], [tx_as * A2R, ty_as * A2R], rtol=1e-12)
    # orthonormal detector frame with u = w x v (u west, v north)
    F = np.stack([w, u, v])
    np.testing.assert_allclose(F @ F.T, np.eye(3), atol=1e-14)
    np.testing.assert_allclose(np.cross(w, v), u, atol=1e-14)


def test_tangent_plane_offsets(ora):
    """One pixel along +column moves by cdelt in theta_x (west) and a row by
    cdelt in theta_y (north), to first order; crota = 90 deg turns +column
    toward north."""
    row, pix = ora.view_from_wcs(215.0, 0.0, 0.0, 0.0, 0.0, 0.0, 3.0, 3.0, 1.0, 1.0, 8, 8)
    d = ora.pixel_direction(row, pix, 1, 0)
    np.testing.assert_allclose(np.arctan2(d[1], -d[0]), 3.0 * A2R, rtol=1e-9)
    rot, _ = ora.view_from_wcs(215.0, 0.0, 0.0, 0.0, 0.0, 90.0, 3.0, 3.0, 1.0, 1.0, 8, 8)
    np.testing.assert_allclose(rot[6:9], [0, 0, 1.0], atol=1e-15)
    np.testing.assert_allclose(rot[9:12], [0, -1.0, 0], atol=1e-15)


def test_synthetic_views_are_wcs_views(ora):
    """The synthetic pinhole views (pointing at the box centre, zero roll)
    are the WCS views with crval = 0, crota = 0."""
    views, pix = ts.make_views([0.0, 45.0, 250.0], (32, 32), 3.2)
    for row in views:
        lon = np.rad2deg(np.arctan2(row[1], row[0]))
        cd_as = row[12] / A2R
        wrow, _ = ora.view_from_wcs(215.0, lon, 0.0, 0.0, 0.0, 0.0, cd_as, cd_as, 16.5, 16.5, 32, 32)
        np.testing.assert_allclose(wrow, row, rtol=1e-12, atol=1e-12)
