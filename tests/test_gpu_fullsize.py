"""The configurations at their real sizes against the FP64 oracle.

* The EUVI-like static inversion (128^3 cube with the unit sphere masked,
  28 views of 512x512, 1% noise, lambda 1e-2): ten CG iterations, the
  residual history and the iterate against the oracle's CG on the same data.
* The COR1-like time-evolving model (8 frames of 256^3 on [-4, 4]^3, 60
  views of 512x512 dealt to the frames unevenly, detector annulus 1.4-4 R_sun
  kept, unit sphere masked): every pixel of P and every voxel of P^T against
  the oracle, and the full batch with its four extra reconstructions in the
  persistent launches against the per-system calls, bit for bit.

Each test prints what it runs before it starts, so that a run that stops
early names its case.
"""
import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import assert_p_close, length_resolution, need_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tomo():
    t = need_gpu()
    t.autotune_clear()
    return t


def _say(msg):
    print(f"[fullsize] {msg}", flush=True)


@pytest.mark.timeout(600)
def test_euvi_cg_matches_oracle(tomo, ora):
    """Ten CG iterations of the EUVI-like inversion, GPU (FP32 vectors, FP64
    scalars, deterministic P^T) against the oracle's FP64 CG on the same
    FP32 data: every entry of the residual history within 2e-4 relative, the
    iterate within 1e-4 in norm and, voxel by voxel, within 1e-3 of the
    oracle iterate's largest value.  Masked voxels stay exactly 0."""
    _say("EUVI-like CG, 10 iterations: oracle data")
    wl = ts.euvi()
    g = wl.geom
    y0 = ora.project(g, wl.x)
    rms = float(np.sqrt(np.mean(y0 * y0)))
    y = (y0 + ts.gaussian_noise(g.nrays, wl.noise_rel * rms, wl.noise_seed)).astype(np.float32)
    y = y.astype(np.float64)
    _say("EUVI-like CG: GPU solve")
    dg = tomo.DeviceGeometry(g)
    x, rep = tomo.cg_solve(dg, to_dev(y), lam_r=wl.lam_r, max_iter=10)
    xg = to_host(x)
    _say("EUVI-like CG: oracle solve")
    xo, ho = ora.cg(ora.normal_operator(g, wl.lam_r), ora.rhs(g, y), n_iter=10)
    assert rep["iters"] == 10 and rep["status"] in (0, tomo.tomo.TOMO_ENOCONV)
    dev_h = np.max(np.abs(rep["history"] / ho - 1.0))
    dev_x = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    dev_v = np.max(np.abs(xg - xo)) / np.max(np.abs(xo))
    _say(f"EUVI-like CG: history {dev_h:.2e}, iterate {dev_x:.2e} (norm), {dev_v:.2e} (per voxel)")
    np.testing.assert_allclose(rep["history"], ho, rtol=2e-4)
    assert dev_x <= 1e-4
    assert dev_v <= 1e-3
    assert np.all(xg[g.map_mask == 0] == 0.0)


@pytest.fixture(scope="module")
def cor1():
    _say("COR1-like: building the 8-frame phantom")
    return ts.cor1_frames()


@pytest.mark.timeout(900)
def test_cor1_projector_matches_oracle(tomo, ora, cor1):
    """Every pixel of P and every voxel of P^T (the deterministic blocked
    strategy the solvers use) on the full COR1-like geometry: 8 x 256^3
    frames, 60 views of 512^2 seen by frames floor(8 s / 30), annulus data
    mask and sphere map mask.  Bounds as everywhere: 1e-5 of P|x| per pixel
    and 1e-4 of P^T|y| per voxel, exact zeros where nothing reaches."""
    g = cor1.geom
    assert g.nframes == 8 and g.nviews == 60 and g.data_mask is not None and g.map_mask is not None
    dg = tomo.DeviceGeometry(g)
    res = length_resolution(g)
    _say("COR1-like P: GPU and oracle")
    x = cor1.x
    img = to_host(tomo.project(dg, to_dev(x)))
    xm = np.abs(x * g.map_mask[None])
    worst = assert_p_close(img, ora.project(g, x), ora.project(g, xm), atol=res * np.abs(x).max(), what="C3 P")
    _say(f"COR1-like P: worst relative error {worst:.2e}")
    del img, xm
    _say("COR1-like P^T: GPU and oracle")
    y = np.random.default_rng(31).normal(size=g.nrays).astype(np.float32).astype(np.float64)
    bp = to_host(tomo.backproject(dg, to_dev(y), strategy=tomo.BP_BLOCKED))
    worst = assert_p_close(bp, ora.backproject(g, y), ora.backproject(g, np.abs(y)), rtol=1e-4,
                           atol=res * np.abs(y).max(), what="C3 P^T")
    _say(f"COR1-like P^T: worst relative error {worst:.2e}")
    assert tomo.binning_spills(dg) == 0
    # masked pixels contribute nothing, masked voxels stay 0
    assert np.all(bp.reshape(g.cube_shape())[:, g.map_mask == 0] == 0.0)


@pytest.mark.timeout(600)
def test_cor1_batch_equals_per_system(tomo, cor1):
    """The COR1-like batch exactly as the benchmark runs it: the 8-frame
    model and the 64^3, 96^3, 128^3 and 192^3 extras in one persistent P and
    one persistent P^T launch, then three graph-captured CG iterations, all
    equal to the per-system calls bit for bit."""
    import torch

    extras = ts.cor1_extras()
    works = [cor1] + extras
    dgs = [tomo.DeviceGeometry(w.geom) for w in works]
    _say("COR1-like batch: launches")
    b = tomo.Batch(dgs)
    xs = [to_dev(w.x) for w in works]
    ys = b.project(xs)
    for k, dg in enumerate(dgs):
        assert torch.equal(ys[k], tomo.project(dg, xs[k])), k
    back = b.backproject(ys)
    for k, dg in enumerate(dgs):
        assert torch.equal(back[k], tomo.backproject(dg, ys[k], strategy=tomo.BP_BLOCKED)), k
    assert b.spills() == 0
    del back
    _say("COR1-like batch: CG")
    lam_t = [w.lam_t for w in works]
    xb, reps = b.cg_solve(ys, lam_r=1e-2, lam_t=lam_t, max_iter=3, check_every=3, use_graph=True)
    for k, dg in enumerate(dgs):
        x1, r1 = tomo.cg_solve(dg, ys[k], lam_r=1e-2, lam_t=lam_t[k], max_iter=3, check_every=3,
                               bp_strategy=tomo.BP_BLOCKED)
        assert torch.equal(xb[k], x1), k
        np.testing.assert_array_equal(reps[k]["history"], r1["history"])
    b.close()
