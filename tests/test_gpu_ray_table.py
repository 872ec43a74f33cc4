"""The blocked P^T reading each ray's set-up from the geometry's ray table
(tomo_tuning.bp_ray_table: a CG solve or a batch sets every ray up once
instead of once per voxel block it crosses) gives the results of the
launches that set the rays up themselves, bit for bit: on frames with data
and map masks, the obstacle variant, ragged views with rays that miss the
box, in tomo_cg_solve (plain and flexible CG) and in batches."""
import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import need_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

SUN = np.array([0.0, 0.0, 0.0, 1.0])


@pytest.fixture(scope="module")
def tomo():
    t = need_gpu()
    t.autotune_clear()
    yield t
    t.autotune_clear()


def _masked_frames():
    g = ts.tiny().geom
    rng = np.random.default_rng(17)
    dm = (rng.uniform(size=g.nrays) > 0.3).astype(np.uint8)
    mm = (rng.uniform(size=g.cube_shape()) > 0.2).astype(np.uint8)
    vf = (np.arange(g.nviews) % 3).astype(np.int32)
    return ts.Geometry(g.n, g.lo, g.hi, g.views, g.npix, vf, 3, data_mask=dm, map_mask=mm)


def _obstacle():
    n, lo, hi = ts.box(16, 1.5)
    views, npix = ts.make_views([0.0, 70.0, 160.0, 280.0], (24, 20), 3.2, lat=15.0, dist=4.0)
    return ts.Geometry(n, lo, hi, views, npix, obstacle=SUN.copy())


def _ragged():
    """Views of uneven shapes whose fields of view reach past the box: some
    rays miss it."""
    n, lo, hi = (20, 13, 9), np.array([-1.3, -0.6, -0.9]), np.array([1.7, 1.1, 0.45])
    rows, pix = [], []
    for lon, (nc, nr), fov in [(10.0, (37, 23), 3.0), (123.0, (5, 70), 2.5), (250.0, (1, 1), 1.0)]:
        r, _ = ts.pinhole_view(ts.observer(lon, 12.0, 40.0), npix=(nc, nr), fov=fov)
        rows.append(r)
        pix.append([nc, nr])
    return ts.Geometry(n, lo, hi, np.array(rows), np.array(pix, dtype=np.int32))


GEOMS = {"tiny": lambda: ts.tiny().geom, "masked_frames": _masked_frames, "obstacle": _obstacle,
         "ragged": _ragged}


def _with_table(tomo, on, f):
    old = tomo.set_tuning(bp_ray_table=1 if on else 0)
    try:
        return f()
    finally:
        tomo.set_tuning(**old)


def _data(g, seed):
    rng = np.random.default_rng(seed)
    y = rng.normal(size=g.nrays)
    y[::7] = 0.0  # rays with nothing to deposit are skipped before their set-up
    return to_dev(y)


@pytest.mark.parametrize("name", sorted(GEOMS))
def test_cg_with_table_equals_cg_without(tomo, name):
    g = GEOMS[name]()
    dg = tomo.DeviceGeometry(g)
    y = _data(g, 3)
    kw = dict(lam_r=1e-2, lam_t=0.5 if g.nframes > 1 else 0.0, max_iter=8, bp_strategy=tomo.BP_BLOCKED)
    x1, r1 = _with_table(tomo, True, lambda: tomo.cg_solve(dg, y, **kw))
    x0, r0 = _with_table(tomo, False, lambda: tomo.cg_solve(dg, y, **kw))
    assert r1["iters"] == r0["iters"] == 8
    np.testing.assert_array_equal(r1["history"], r0["history"])
    np.testing.assert_array_equal(to_host(x1), to_host(x0))


def test_flexible_cg_and_graph_mode_with_table(tomo):
    import torch

    from paper_1103_5904_amd import precond as pc

    g = ts.tiny().geom
    dg = tomo.DeviceGeometry(g)
    y = _data(g, 4)
    net = torch.as_tensor(pc.identity_params(1.0).astype(np.float32)).cuda()
    for kw in (dict(precond=net), dict(use_graph=True, check_every=4)):
        x1, r1 = _with_table(tomo, True, lambda: tomo.cg_solve(dg, y, lam_r=1e-2, max_iter=8, **kw))
        x0, r0 = _with_table(tomo, False, lambda: tomo.cg_solve(dg, y, lam_r=1e-2, max_iter=8, **kw))
        np.testing.assert_array_equal(r1["history"], r0["history"])
        np.testing.assert_array_equal(to_host(x1), to_host(x0))


def test_workspace_holds_the_table(tomo):
    g = ts.tiny().geom
    dg = tomo.DeviceGeometry(g)
    with_t = _with_table(tomo, True, lambda: tomo.cg_workspace_bytes(dg, max_iter=10))
    without = _with_table(tomo, False, lambda: tomo.cg_workspace_bytes(dg, max_iter=10))
    table = 11 * 8 * g.nrays + 8 * g.nrays  # eleven FP64 columns and one index word per pixel
    assert table <= with_t - without <= table + 512
    # the solve in exactly that workspace, with the table
    import torch

    ws = torch.empty(with_t, dtype=torch.uint8, device="cuda")
    y = _data(g, 5)
    x1, _ = _with_table(tomo, True, lambda: tomo.cg_solve(dg, y, lam_r=1e-2, max_iter=10, workspace=ws))
    x0, _ = _with_table(tomo, False, lambda: tomo.cg_solve(dg, y, lam_r=1e-2, max_iter=10))
    np.testing.assert_array_equal(to_host(x1), to_host(x0))


def test_batch_with_tables_equals_batch_without(tomo):
    geoms = [GEOMS[k]() for k in sorted(GEOMS)]
    dgs = [tomo.DeviceGeometry(g) for g in geoms]
    ys = [_data(g, 10 + k) for k, g in enumerate(geoms)]
    out = {}
    for on in (True, False):
        b = _with_table(tomo, on, lambda: tomo.Batch(dgs))
        try:
            bp = [to_host(v) for v in b.backproject(ys)]
            xs, reps = b.cg_solve(ys, lam_r=1e-2, max_iter=6)
            out[on] = (bp, [to_host(x) for x in xs], [r["history"] for r in reps])
        finally:
            b.close()
    for k in range(len(geoms)):
        np.testing.assert_array_equal(out[True][0][k], out[False][0][k])
        np.testing.assert_array_equal(out[True][1][k], out[False][1][k])
        np.testing.assert_array_equal(out[True][2][k], out[False][2][k])
    # and the per-system P^T that sets rays up itself
    for k, dg in enumerate(dgs):
        np.testing.assert_array_equal(out[True][0][k], to_host(tomo.backproject(dg, ys[k], strategy=tomo.BP_BLOCKED)))
