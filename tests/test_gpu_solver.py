"""GPU prior and conjugate-gradient solver against the FP64 oracle."""
import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import need_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tomo():
    return need_gpu()


def test_prior_parity(tomo, ora):
    """lambda_r D^T D x + lambda_t D_t^T D_t x on a ragged 3-frame grid: FP32
    stencil vs FP64 (6 terms of O(|x|) each: relative 1e-6 of the sum of
    absolute terms)."""
    n = (11, 7, 5)
    dg = tomo.DeviceGeometry(ts.Geometry(n, np.zeros(3), np.ones(3), ts.make_views([0.0], (1, 1), 1.0)[0],
                                         np.array([[1, 1]], np.int32), np.zeros(1, np.int32), 3))
    x = np.random.default_rng(0).normal(size=dg.cube_shape)
    xf = x.astype(np.float32).astype(np.float64)
    got = to_host(tomo.apply_prior(dg, to_dev(xf), 0.3, 2.0))
    ref = 0.3 * ora.laplacian6(xf) + 2.0 * ora.laplacian_t(xf)
    scale = 0.3 * 12 * np.abs(xf).max() + 2.0 * 4 * np.abs(xf).max()
    assert np.max(np.abs(got - ref)) <= 1e-6 * scale


def _tiny_problem(ora):
    wl = ts.tiny()
    y = ora.project(wl.geom, wl.x).astype(np.float32).astype(np.float64)
    return wl, y


def test_cg_tiny_matches_oracle(tomo, ora):
    """Twenty CG iterations on the tiny problem: GPU (FP32 vectors, FP64
    scalars) vs the FP64 oracle, iterate by iterate through the residual
    history and at the final x."""
    wl, y = _tiny_problem(ora)
    dg = tomo.DeviceGeometry(wl.geom)
    x, rep = tomo.cg_solve(dg, to_dev(y), lam_r=wl.lam_r, max_iter=20)
    xg = to_host(x)
    A = ora.normal_operator(wl.geom, wl.lam_r)
    xo, ho = ora.cg(A, ora.rhs(wl.geom, y), n_iter=20)
    assert rep["iters"] == 20 and rep["status"] == 0
    np.testing.assert_allclose(rep["history"], ho, rtol=2e-4)
    assert np.linalg.norm(xg - xo) <= 1e-4 * np.linalg.norm(xo)
    # the recursive residual tracks the true one
    assert abs(rep["true_rel_res"] - rep["rel_res"]) <= 1e-3 * rep["rel_res"] + 1e-6


def test_cg_masked_temporal_matches_oracle(tomo, ora):
    """Three frames coupled by the temporal prior, map mask on: 15 iterations."""
    wl = ts.tiny()
    g0 = wl.geom
    vf = (np.arange(g0.nviews) % 3).astype(np.int32)
    mm = ts.sphere_map_mask(g0.n, g0.lo, g0.hi, 0.6)
    g = ts.Geometry(g0.n, g0.lo, g0.hi, g0.views, g0.npix, vf, 3, None, mm)
    x = np.stack([wl.x * (1 + 0.1 * f) for f in range(3)])
    y = ora.project(g, x).astype(np.float32).astype(np.float64)
    dg = tomo.DeviceGeometry(g)
    xg, rep = tomo.cg_solve(dg, to_dev(y), lam_r=1e-2, lam_t=10.0, max_iter=15)
    xg = to_host(xg)
    xo, ho = ora.cg(ora.normal_operator(g, 1e-2, 10.0), ora.rhs(g, y), n_iter=15)
    np.testing.assert_allclose(rep["history"], ho, rtol=2e-4)
    assert np.linalg.norm(xg - xo) <= 1e-4 * np.linalg.norm(xo)
    assert np.all(xg[:, mm == 0] == 0.0)


def test_cg_stops_at_rtol(tomo, ora):
    wl, y = _tiny_problem(ora)
    dg = tomo.DeviceGeometry(wl.geom)
    x, rep = tomo.cg_solve(dg, to_dev(y), lam_r=wl.lam_r, max_iter=500, rtol=1e-3, check_every=4)
    assert rep["status"] == 0
    assert rep["rel_res"] <= 1e-3
    assert rep["true_rel_res"] <= 1e-3
    h = rep["history"]
    assert len(h) == rep["iters"] + 1 and h[-2] > 1e-3  # stopped at the first iterate below


def test_cg_warm_start(tomo, ora):
    wl, y = _tiny_problem(ora)
    dg = tomo.DeviceGeometry(wl.geom)
    x1, r1 = tomo.cg_solve(dg, to_dev(y), lam_r=wl.lam_r, max_iter=10)
    x2, r2 = tomo.cg_solve(dg, to_dev(y), x0=x1, lam_r=wl.lam_r, max_iter=10)
    assert r2["history"][0] == pytest.approx(r1["true_rel_res"], rel=1e-3)
    assert r2["rel_res"] < r1["rel_res"]


def test_cg_reports_non_finite(tomo, ora):
    """A NaN in a pixel whose ray crosses the cube poisons b = P^T y: the
    solver must stop and say so instead of iterating on NaNs."""
    wl, y = _tiny_problem(ora)
    y[16 * 32 + 16] = np.nan  # view 0, central pixel
    dg = tomo.DeviceGeometry(wl.geom)
    _, rep = tomo.cg_solve(dg, to_dev(y), lam_r=wl.lam_r, max_iter=5)
    assert rep["status"] == tomo.tomo.TOMO_ENONFINITE


def test_cg_euvi_full(tomo):
    """The EUVI-like inversion (28 views of 512^2, 128^3, 50 iterations): the
    recursive residual falls steadily and agrees with the true residual."""
    import torch

    wl = ts.euvi()
    dg = tomo.DeviceGeometry(wl.geom)
    y0 = tomo.project(dg, to_dev(wl.x))
    rms = float(torch.sqrt(torch.mean(y0.double() ** 2)))
    y = y0 + to_dev(ts.gaussian_noise(wl.geom.nrays, wl.noise_rel * rms, wl.noise_seed))
    x, rep = tomo.cg_solve(dg, y, lam_r=wl.lam_r, max_iter=50, time_kernels=True)
    h = rep["history"]
    assert rep["iters"] == 50 and len(h) == 51
    assert h[-1] < 0.05 * h[0]
    assert abs(rep["true_rel_res"] - rep["rel_res"]) <= 0.05 * rep["rel_res"]
    assert rep["ms_project"] > 0 and rep["ms_backproject"] > 0
    xm = to_host(x)
    assert np.all(xm[wl.geom.map_mask == 0] == 0.0)
