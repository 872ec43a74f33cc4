"""GPU parity at the sizes of the paper's projector scaling sweeps
(Sec. "Performance", the image-size and cube-size tables): 64 images, no
mask and no obstacle, up to 1024^2 images on a 128^3 cube and a 1024^3 cube
(2^30 voxels, 4 GiB, the largest frame the library takes) under 256^2
images.  P on sampled pixels and P^T on sampled voxels against the oracle's
Siddon traces (values of the separable phantom recomputed at each voxel),
the crossing count against the oracle's exact count, and adjointness over
the whole operator."""
import numpy as np
import pytest
import torch

import tomo_synth as ts
from _gpu_common import CODES, P_RTOL, PT_RTOL, assert_p_close, length_resolution, need_gpu, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tomo():
    return need_gpu()


def _case(tomo, n, npix):
    g = ts.sweep_geometry(n, npix)
    parts = ts.sweep_cube_parts(n)
    dg = tomo.DeviceGeometry(g)
    x = torch.as_tensor(ts.sweep_cube(parts)).cuda()
    return g, parts, dg, x


def _sampled_p(ora, g, parts, img, count, seed):
    rng = np.random.default_rng(seed)
    off = g.view_offsets()
    got, want, wabs = [], [], []
    for _ in range(count):
        v = int(rng.integers(0, g.nviews))
        ncol, nrow = (int(t) for t in g.npix[v])
        c, r = int(rng.integers(0, ncol)), int(rng.integers(0, nrow))
        d = ora.pixel_direction(g.views[v], g.npix[v], c, r)
        idx, ln, _ = ora.trace_ray(g.n, g.lo, g.hi, g.views[v][0:3], d)
        xv = ts.sweep_values(parts, idx).astype(np.float64)
        got.append(img[off[v] + r * ncol + c])
        want.append(float(np.sum(ln * xv)))
        wabs.append(float(np.sum(ln * np.abs(xv))))
    return np.array(got), np.array(want), np.array(wabs)


def _voxel_pt(ora, g, y, vox):
    """(P^T y)_vox and (P^T |y|)_vox from the oracle traces of every pixel
    whose ray can cross the voxel: the bounding rectangle of the voxel's
    eight corners projected on each detector, widened by one pixel."""
    nx, ny, nz = g.n
    i, j, k = vox % nx, (vox // nx) % ny, vox // (nx * ny)
    dlt = (g.hi - g.lo) / np.array(g.n, dtype=np.float64)
    corners = np.array([g.lo + (np.array([i + a, j + b, k + c]) * dlt)
                        for a in (0, 1) for b in (0, 1) for c in (0, 1)])
    off = g.view_offsets()
    s = sa = 0.0
    for v in range(g.nviews):
        row = g.views[v]
        o, w, u, vv, cd, cp = row[0:3], row[3:6], row[6:9], row[9:12], row[12:14], row[14:16]
        ncol, nrow = (int(t) for t in g.npix[v])
        rel = corners - o
        depth = rel @ w
        assert np.all(depth > 0)
        cols = cp[0] + (rel @ u) / depth / cd[0]
        rows = cp[1] + (rel @ vv) / depth / cd[1]
        c0, c1 = max(int(np.floor(cols.min())) - 1, 0), min(int(np.ceil(cols.max())) + 1, ncol - 1)
        r0, r1 = max(int(np.floor(rows.min())) - 1, 0), min(int(np.ceil(rows.max())) + 1, nrow - 1)
        for r in range(r0, r1 + 1):
            for c in range(c0, c1 + 1):
                d = ora.pixel_direction(row, g.npix[v], c, r)
                idx, ln, _ = ora.trace_ray(g.n, g.lo, g.hi, o, d)
                hit = ln[idx == vox]
                if hit.size:
                    yy = float(y[off[v] + r * ncol + c])
                    s += float(hit.sum()) * yy
                    sa += float(hit.sum()) * abs(yy)
    return s, sa


def _check(tomo, ora, n, npix, n_pix, n_vox, seed):
    g, parts, dg, x = _case(tomo, n, npix)
    img = to_host(tomo.project(dg, x))
    res = length_resolution(g)
    got, want, wabs = _sampled_p(ora, g, parts, img, n_pix, seed)
    assert_p_close(got, want, wabs, rtol=P_RTOL, atol=res * 1.5)
    rng = np.random.default_rng(seed + 1)
    y = rng.normal(size=g.nrays).astype(np.float32)
    yd = torch.as_tensor(y).cuda()
    bt = tomo.backproject(dg, yd, strategy=CODES["blocked"])
    voxels = rng.integers(0, g.nvox, size=n_vox)
    btv = bt.reshape(-1)[torch.as_tensor(voxels).cuda()].double().cpu().numpy()
    ref = np.array([_voxel_pt(ora, g, y, int(v)) for v in voxels])
    # rays are sparser than voxels at the largest cube (a 256^2 pixel is 4
    # voxels wide), so some sampled voxels are crossed by no ray
    assert np.count_nonzero(ref[:, 1]) >= 0.5 * n_vox
    assert_p_close(btv, ref[:, 0], ref[:, 1], rtol=PT_RTOL, what="P^T", atol=res * float(np.abs(y).max()))
    # <P x, y> = <x, P^T y> over the whole operator (FP64 sums on the GPU)
    lhs = float(torch.dot(torch.as_tensor(img).cuda(), yd.double()))
    rhs = float(torch.dot(x.reshape(-1).double(), bt.reshape(-1).double()))
    scale = float(torch.dot(torch.as_tensor(np.abs(img)).cuda(), yd.double().abs()))
    assert abs(lhs - rhs) <= 1e-5 * scale
    return g, dg


def test_images_1024_on_128_cube(tomo, ora):
    """64 views of 1024^2 on the 128^3 cube (the image-size table's largest
    point): 2000 pixels, 12 voxels."""
    _check(tomo, ora, 128, 1024, 2000, 12, 60)


def test_cube_512(tomo, ora):
    _check(tomo, ora, 512, 256, 1500, 40, 61)


def test_cube_1024(tomo, ora):
    """2^30 voxels (4 GiB) under 64 views of 256^2 (the cube-size table's
    largest point): sampled P and P^T, the exact crossing count, and the
    atomic strategies' refusal of such a frame."""
    g, dg = _check(tomo, ora, 1024, 256, 1500, 40, 62)
    assert tomo.count_crossings(dg) == ora.count_crossings(g)
    y = torch.zeros(g.nrays, dtype=torch.float32, device="cuda")
    for strat in ("binned", "atomic"):
        with pytest.raises(tomo.TomoError):
            tomo.backproject(dg, y, strategy=CODES[strat])


def test_autotune_is_never_slower(tomo):
    """The tuner keeps a candidate only if it beats the process-wide tuning
    in alternation through the same launch paths, so on a sweep point where
    an earlier tuner picked a slower back-projection (128^3 under 128^2)
    the tuned launches are at most 2% slower than the default ones, timed
    here in alternation (medians of five rounds of 20 launches)."""
    g, parts, dg, x = _case(tomo, 128, 128)
    y = tomo.project(dg, x)
    out = torch.empty_like(x)

    def per_launch(f, n=20):
        f()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            f()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / n

    default = tomo.get_tuning()
    tomo.autotune_clear()
    tomo.autotune(dg, reps=5)
    tuned, is_tuned = tomo.class_tuning(dg)
    assert is_tuned
    tomo.autotune_clear()
    times = {"P": ([], []), "P^T": ([], [])}
    try:
        for _ in range(5):
            for key, f in (("P", lambda: tomo.project(dg, x, out=y)), ("P^T", lambda: tomo.backproject(dg, y, out=out))):
                tomo.set_tuning(**tuned)
                times[key][0].append(per_launch(f))
                tomo.set_tuning(**default)
                times[key][1].append(per_launch(f))
    finally:
        tomo.set_tuning(**default)
    for key, (tt, td) in times.items():
        print(f"{key}: tuned {np.median(tt):.4f} ms, default {np.median(td):.4f} ms", flush=True)
        assert np.median(tt) <= 1.02 * np.median(td), key
