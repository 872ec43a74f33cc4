"""Batched persistent launches and the autotuner: the batch's single P and
P^T launches over uneven systems equal the per-system calls bit for bit,
the batched CG (with and without graph capture) equals the per-system CG,
and autotuned launches keep oracle parity."""
import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import assert_p_close, length_resolution, need_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tomo():
    t = need_gpu()
    yield t
    t.autotune_clear()


def _ragged():
    n, lo, hi = (20, 13, 9), np.array([-1.3, -0.6, -0.9]), np.array([1.7, 1.1, 0.45])
    rows, pix = [], []
    for lon, (nc, nr), fov in [(10.0, (37, 23), 3.0), (123.0, (5, 70), 2.5), (250.0, (1, 1), 1.0)]:
        r, _ = ts.pinhole_view(ts.observer(lon, 12.0, 40.0), npix=(nc, nr), fov=fov)
        rows.append(r)
        pix.append([nc, nr])
    return ts.Geometry(n, lo, hi, np.array(rows), np.array(pix, dtype=np.int32))


def _masked_frames():
    g = ts.tiny().geom
    rng = np.random.default_rng(7)
    dm = (rng.uniform(size=g.nrays) > 0.3).astype(np.uint8)
    mm = (rng.uniform(size=g.cube_shape()) > 0.2).astype(np.uint8)
    vf = (np.arange(g.nviews) % 3).astype(np.int32)
    return ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, vf, 3, data_mask=dm, map_mask=mm)


def _systems():
    return [ts.tiny().geom, _masked_frames(), _ragged(), ts.euvi(64, 128).geom.subset([0, 9, 20])]


def test_batched_projections_equal_per_system_calls(tomo):
    import torch

    geoms = _systems()
    dgs = [tomo.DeviceGeometry(g) for g in geoms]
    b = tomo.Batch(dgs)
    assert b.items(0) == sum(-(-int(c) // 16) * -(-int(r) // 16) for g in geoms for c, r in g.npix)
    rng = np.random.default_rng(3)
    cubes = [to_dev(rng.uniform(size=dg.cube_shape)) for dg in dgs]
    imgs = [to_dev(rng.normal(size=dg.npix)) for dg in dgs]
    for rep in range(2):  # the second launch checks that the work queues reset themselves
        got_p = b.project(cubes)
        got_b = b.backproject(imgs)
        torch.cuda.synchronize()
        for k, dg in enumerate(dgs):
            assert torch.equal(got_p[k], tomo.project(dg, cubes[k])), (rep, k)
            assert torch.equal(got_b[k], tomo.backproject(dg, imgs[k], strategy=tomo.BP_BLOCKED)), (rep, k)
    acc = [c.clone() for c in cubes]
    b.backproject(imgs, outs=acc, accumulate=True)
    for k, dg in enumerate(dgs):
        ref = cubes[k].clone()
        tomo.backproject(dg, imgs[k], out=ref, accumulate=True, strategy=tomo.BP_BLOCKED)
        assert torch.equal(acc[k], ref), k
    assert b.spills() == 0


def test_batched_projections_match_the_oracle(tomo, ora):
    geoms = _systems()[:3]
    dgs = [tomo.DeviceGeometry(g) for g in geoms]
    b = tomo.Batch(dgs)
    rng = np.random.default_rng(4)
    xs = [rng.uniform(size=g.cube_shape()) for g in geoms]
    ys = [rng.normal(size=g.nrays) for g in geoms]
    got_p = b.project([to_dev(x) for x in xs])
    got_b = b.backproject([to_dev(y) for y in ys])
    for k, g in enumerate(geoms):
        res = length_resolution(g)
        mm = 1.0 if g.map_mask is None else (g.map_mask if g.nframes == 1 else g.map_mask[None])
        assert_p_close(to_host(got_p[k]), ora.project(g, xs[k]), ora.project(g, np.abs(xs[k] * mm)),
                       atol=res * np.abs(xs[k]).max())
        assert_p_close(to_host(got_b[k]), ora.backproject(g, ys[k]), ora.backproject(g, np.abs(ys[k])),
                       rtol=1e-4, what=f"P^T system {k}", atol=res * np.abs(ys[k]).max())


def _data(tomo, dgs, geoms, seed):
    rng = np.random.default_rng(seed)
    ys = []
    for dg, g in zip(dgs, geoms):
        x = rng.uniform(size=g.cube_shape())
        ys.append(tomo.project(dg, to_dev(x)))
    return ys


@pytest.mark.parametrize("use_graph", [False, True])
def test_batched_cg_equals_per_system_cg(tomo, use_graph):
    """Each system with its own weights, limits and tolerance: iterates,
    histories and reports equal the single-system solver's (same kernels,
    blocked P^T) exactly."""
    import torch

    geoms = _systems()[:3]
    dgs = [tomo.DeviceGeometry(g) for g in geoms]
    ys = _data(tomo, dgs, geoms, 5)
    lam_r, lam_t, max_iter, rtol = [1e-2, 3e-2, 1e-2], [0.0, 5.0, 0.0], [12, 30, 7], [0.0, 2e-3, 0.0]
    b = tomo.Batch(dgs)
    xs, reps = b.cg_solve(ys, lam_r=lam_r, lam_t=lam_t, max_iter=max_iter, rtol=rtol, check_every=4,
                          use_graph=use_graph)
    for k, dg in enumerate(dgs):
        x1, r1 = tomo.cg_solve(dg, ys[k], lam_r=lam_r[k], lam_t=lam_t[k], max_iter=max_iter[k], rtol=rtol[k],
                               check_every=4, bp_strategy=tomo.BP_BLOCKED)
        assert torch.equal(xs[k], x1), k
        np.testing.assert_array_equal(reps[k]["history"], r1["history"])
        for key in ("iters", "status", "n_project", "n_backproject"):
            assert reps[k][key] == r1[key], (k, key)
        assert reps[k]["true_rel_res"] == r1["true_rel_res"]
    assert reps[1]["status"] == 0 and reps[1]["iters"] < 30  # converged on its own tolerance


def test_batched_cg_kernel_timing(tomo):
    """time_kernels in a batched solve, replayed from a graph (the events
    are graph nodes) and enqueued directly: the same iterates either way,
    positive P and P^T totals shared by every report, and per launch within
    a factor 3 of each other (the two runs time the same launches)."""
    import torch

    geoms = _systems()[:3]
    dgs = [tomo.DeviceGeometry(g) for g in geoms]
    ys = _data(tomo, dgs, geoms, 12)
    b = tomo.Batch(dgs)
    out = {}
    for use_graph in (True, False):
        xs, reps = b.cg_solve(ys, lam_r=1e-2, max_iter=8, check_every=4, use_graph=use_graph, time_kernels=True)
        out[use_graph] = ([x.clone() for x in xs], reps)
        for r in reps:
            assert r["ms_project"] == reps[0]["ms_project"] > 0.0
            assert r["ms_backproject"] == reps[0]["ms_backproject"] > 0.0
    for a, c in zip(out[True][0], out[False][0]):
        assert torch.equal(a, c)
    for key in ("ms_project", "ms_backproject"):
        ratio = out[True][1][0][key] / out[False][1][0][key]
        assert 1 / 3 < ratio < 3, (key, ratio)
    _, reps = b.cg_solve(ys, lam_r=1e-2, max_iter=8, check_every=4, use_graph=True)
    assert reps[0]["ms_project"] == 0.0 and reps[0]["ms_backproject"] == 0.0


def test_single_solver_graph_mode(tomo):
    import torch

    g = ts.tiny().geom
    dg = tomo.DeviceGeometry(g)
    y = _data(tomo, [dg], [g], 6)[0]
    x0 = to_dev(np.random.default_rng(8).uniform(size=g.cube_shape()))
    a, ra = tomo.cg_solve(dg, y, x0, lam_r=1e-2, max_iter=15, check_every=5, use_graph=True)
    c, rc = tomo.cg_solve(dg, y, x0, lam_r=1e-2, max_iter=15, check_every=5, bp_strategy=tomo.BP_BLOCKED)
    assert torch.equal(a, c)
    np.testing.assert_array_equal(ra["history"], rc["history"])


def test_cor1_like_batch(tomo):
    """A reduced COR1-like batch: three 48^3 time frames on [-4, 4]^3 with
    the unit sphere masked, the detector annulus 1.4-4 kept and a temporal
    prior, plus two independent reconstructions of other sizes, solved
    together; each system equals its own solve."""
    import torch

    wl = ts.cor1_frames(n=48, K=3, npix=64, nsteps=6)
    extras = [ts.Geometry(*ts.box(n, 1.5), *ts.make_views([30.0 * k for k in range(6)], (48, 48), 3.4))
              for n in (24, 40)]
    geoms = [wl.geom] + extras
    dgs = [tomo.DeviceGeometry(g) for g in geoms]
    ys = [tomo.project(dgs[0], to_dev(wl.x))] + _data(tomo, dgs[1:], extras, 9)
    b = tomo.Batch(dgs)
    lam_t = [10.0, 0.0, 0.0]
    xs, reps = b.cg_solve(ys, lam_r=1e-2, lam_t=lam_t, max_iter=10, check_every=5, use_graph=True)
    for k, dg in enumerate(dgs):
        x1, _ = tomo.cg_solve(dg, ys[k], lam_r=1e-2, lam_t=lam_t[k], max_iter=10, check_every=5,
                              bp_strategy=tomo.BP_BLOCKED)
        assert torch.equal(xs[k], x1), k
        assert reps[k]["iters"] == 10


def test_autotune_keeps_parity(tomo, ora):
    g = ts.tiny().geom
    dg = tomo.DeviceGeometry(g)
    chosen = tomo.autotune(dg, reps=2)
    now, tuned = tomo.class_tuning(dg)
    assert tuned and now == chosen
    assert chosen["bp_default"] in (1, 2, 3)
    x = np.random.default_rng(10).uniform(size=g.cube_shape())
    y = np.random.default_rng(11).normal(size=g.nrays)
    res = length_resolution(g)
    assert_p_close(to_host(tomo.project(dg, to_dev(x))), ora.project(g, x), ora.project(g, np.abs(x)),
                   atol=res * np.abs(x).max())
    assert_p_close(to_host(tomo.backproject(dg, to_dev(y))), ora.backproject(g, y), ora.backproject(g, np.abs(y)),
                   rtol=1e-4, what="P^T after autotune", atol=res * np.abs(y).max())
    tomo.autotune_clear()
    assert not tomo.class_tuning(dg)[1]
