"""The allocation-free transpose (tomo_backproject_noalloc) against the
allocating one (tomo_backproject_ex with the blocked strategy), through the
C ABI: bit for bit on two calls in a row, the second with a smaller input,
and the two refusals (a geometry without device tables; scratch beyond the
static array)."""
import numpy as np
import pytest

import tomo_synth as ts
from _gpu_common import need_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tomo():
    t = need_gpu()
    t.autotune_clear()
    return t


def _check_equal(tomo, g, seed, accumulate=False):
    import torch

    dg = tomo.DeviceGeometry(g)
    tomo.count_crossings(dg)  # builds the geometry's device tables
    y = to_dev(np.random.default_rng(seed).normal(size=dg.npix))
    base = to_dev(np.random.default_rng(seed + 1).uniform(size=dg.cube_shape))
    ref = base.clone()
    tomo.backproject(dg, y, out=ref, accumulate=accumulate, strategy=tomo.BP_BLOCKED)
    got = torch.full_like(base, float("nan")) if not accumulate else base.clone()
    tomo.backproject_noalloc(dg, y, got, accumulate=accumulate)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)


def test_noalloc_equals_blocked_backprojection(tomo):
    """First a 128^3 EUVI-like geometry with 28 views of 256^2 (four owners per
    block: 32 MiB of partial sums in the static array), then the 32^3 tiny
    geometry (one owner), then the first again with accumulate: each equal
    to the allocating call."""
    big = ts.euvi(128, 256).geom
    print("[noalloc] 128^3, 28 x 256^2", flush=True)
    _check_equal(tomo, big, 1)
    print("[noalloc] 32^3, 8 x 32^2", flush=True)
    _check_equal(tomo, ts.tiny().geom, 2)
    print("[noalloc] 128^3 again, accumulate", flush=True)
    _check_equal(tomo, big, 3, accumulate=True)


def test_noalloc_refusals(tomo):
    import torch

    g = ts.tiny(5).geom
    g.views[0, 0] += 1e-3  # a geometry no call has used yet
    dg = tomo.DeviceGeometry(g)
    y = torch.zeros(dg.npix, dtype=torch.float32, device="cuda")
    out = torch.zeros(dg.cube_shape, dtype=torch.float32, device="cuda")
    with pytest.raises(tomo.TomoError):
        tomo.backproject_noalloc(dg, y, out)
    # eight owners per block over a 128^3 cube need 64 MiB of partial sums
    # plus the per-view maxima: more than the static array
    before = tomo.get_tuning()
    try:
        tomo.set_tuning(bp_splits=8)
        g2 = ts.euvi(128, 64).geom
        dg2 = tomo.DeviceGeometry(g2)
        tomo.count_crossings(dg2)
        y2 = torch.zeros(dg2.npix, dtype=torch.float32, device="cuda")
        out2 = torch.zeros(dg2.cube_shape, dtype=torch.float32, device="cuda")
        with pytest.raises(tomo.TomoError):
            tomo.backproject_noalloc(dg2, y2, out2)
    finally:
        tomo.set_tuning(**before)
