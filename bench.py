"""Benchmark: Siddon P / P^T voxel-crossings per second on one MI355X.

One step is the EUVI-like static inversion: 50 conjugate-gradient
iterations on the 128^3 cube (unit sphere masked) seen by 28 views of
512x512 pixels, i.e. one P^T for the right-hand side, then per iteration one
P, one P^T, the prior and the vector updates, plus one P and P^T for the
final true residual.  Inputs (phantom, data with 1% noise) are synthetic,
generated once and resident in HBM before timing.

value = (P and P^T applications in the step) x (voxel crossings per
application) / step time.  The roofline entry is for the kernel that takes
most of the step time, timed per launch with HIP events recorded on the
stream the library launches it on.  Next to it, the achieved algorithmic
bandwidth as a fraction of device copies that stream from HBM and from the
Infinity Cache (achievable), and the crossing rate as a fraction of the VALU
ceiling of the walk loops' instruction counts (valu).  The CPU baseline is the
FP64 oracle on a bounded sample of the same workload.  After the timed steps,
the learned preconditioner's wall time to relative residual 1e-3 is compared
with plain CG on held-out problems of its own family (time_to_rel_res_1e-3),
and the
COR1-like batch (five systems of uneven size in persistent launches with
autotuned shapes) is timed against solving its systems one after another
(batched), the obstacle variant (lines of sight ending at the photosphere)
is measured on the headline workload (obstacle), the Thomson-scattering
operators pB and B on a COR1-like frame (thomson), the headline workload
as two instruments with gains and the height-weighted prior (height_gain),
P and P^T on the other configurations' geometries (configs), and the
paper's image-size and cube-size projector sweeps (sweep).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Siddon P/Pᵀ voxel-crossings/s; time to rel. residual 1e-3 (learned vs plain)"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE passes on this workload (scaled by a
# 256 MiB copy's counts; profiles/euvi128_cg50_blocked_backprojection.md), valid only for the kernel
# sources and default launch shapes (api.hip) they were taken on: sha256 over the listed files, first
# 16 hex digits.
TRAFFIC = {
    "k_backproject_blocked": (158.4e6, "09199c508949126a",
                              ["blocked.h", "blocked.hip", "walk.h", "common.h", "api.hip"]),
    "k_project": (264.4e6, "870940f8054ca25a", ["siddon.hip", "walk.h", "common.h", "api.hip"]),
}


# VALU instructions per voxel crossing in the walk loops of the built gfx950
# code (one loop step per crossing: the min of four crossing parameters, the
# segment length, tie tests and FMA updates of the three axes, the offset
# advance, and the gather (P) or the fixed-point LDS deposit (P^T)), read from
# `hipcc --cuda-device-only -S` of siddon.hip and blocked.hip; the set-ups are
# not counted.  With FP64 at the full wave64 rate, the chip issues 256 CUs x 64
# lanes x 2.4 GHz = 39.3e12 such instructions per second.
VALU_PER_CROSSING = {"k_project": 21, "k_backproject_blocked": 23}
VALU_LANE_RATE = 256 * 64 * 2.4e9


def probes(reps=5):
    """Achievable bandwidths measured with plain device copies (torch): a
    2 GiB buffer (HBM; the cube and images of the headline are far smaller)
    and a 32 MiB buffer copied 20 times over (resident in the 256 MB Infinity
    Cache).  Bytes read + written per second, median of `reps`."""
    import torch

    def rate(nbytes, inner):
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(inner):
                dst.copy_(src)
            e1.record()
            e1.synchronize()
            t.append(e0.elapsed_time(e1))
        del src, dst
        torch.cuda.empty_cache()
        return 2.0 * nbytes * inner / (float(np.median(t)) * 1e-3) / 1e9

    return {"hbm_copy_gbs": rate(2 << 30, 1), "mall_copy_gbs": rate(32 << 20, 20)}


def measured_traffic(kernel):
    """The profiled HBM bytes of `kernel`, or None if its sources changed since."""
    import hashlib

    if kernel not in TRAFFIC:
        return None
    nbytes, digest, files = TRAFFIC[kernel]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1103_5904_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return nbytes if digest is not None and h.hexdigest()[:16] == digest else None


def log(msg):
    """Progress on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=6,
                    help="full P + P^T passes of the oracle in its timed sample")
    ap.add_argument("--bp", choices=["auto", "blocked", "binned", "atomic"], default="auto",
                    help="back-projection strategy")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-plain time to relative residual 1e-3")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched COR1-like measurement")
    ap.add_argument("--no-obstacle", action="store_true",
                    help="skip the obstacle-variant measurement")
    ap.add_argument("--no-thomson", action="store_true",
                    help="skip the Thomson-scattering operator measurement")
    ap.add_argument("--no-height-gain", action="store_true",
                    help="skip the two-instrument, height-weighted-prior measurement")
    ap.add_argument("--no-probes", action="store_true",
                    help="skip the device-copy bandwidth probes (they share the copy kernel that "
                         "calibrates the byte counters)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip P and P^T on the other configurations' geometries")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the paper's image-size and cube-size projector sweeps")
    ap.add_argument("--sweep-only", type=int, nargs=2, metavar=("CUBE", "IMAGE"), default=None,
                    help="run only the sweep point with this cube side and image side, and print "
                         "its line (for profiling it alone)")
    ap.add_argument("--sweep-no-autotune", action="store_true",
                    help="time the sweep with the default launch shapes only")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="before the timed steps, run 3 device-to-device copies of MIB MiB: the "
                         "known-size kernel that calibrates hardware byte counters")
    return ap.parse_args()


def learned_vs_plain(tomo, ts, seeds=tuple(range(2003, 2013)), reps=3):
    """Wall time from tomo_cg_solve entry to a confirmed true relative
    residual <= 1e-3 on held-out learned-preconditioner problems (128^3 blob
    phantom, 28 views of 256x256, 1% noise, lambda 1e-2; the shipped network
    was trained on seeds 1000-1049, and seeds 2000-2002 informed its recipe):
    plain CG against flexible CG with the network, median of `reps` after one
    warm-up each per problem, then the median over the ten problems."""
    import torch

    from paper_1103_5904_amd import precond as pc

    net = pc.load(os.path.join(ROOT, "paper_1103_5904_amd", "precond_weights.npz"))
    rows = []
    for seed in seeds:
        wl = ts.learned(seed)
        dg = tomo.DeviceGeometry(wl.geom)
        y = pc.noisy_data(dg, torch.as_tensor(wl.x.astype(np.float32)).cuda(), wl.noise_rel,
                          wl.noise_seed)
        res = {"seed": seed}
        for name, params in (("plain", None), ("learned", net)):
            pc.time_to_tolerance(dg, y, wl.lam_r, 1e-3, params)
            ms, rep = pc.time_to_tolerance(dg, y, wl.lam_r, 1e-3, params, reps=reps)
            res[f"{name}_ms"] = ms
            res[f"{name}_iters"] = rep["iters"]
            res[f"{name}_true_rel_res"] = rep["true_rel_res"]
        res["speedup"] = res["plain_ms"] / res["learned_ms"]
        rows.append(res)
    return {"rtol": 1e-3, "workload": "128^3 blob phantom, 28 views of 256x256, 1% noise, "
                                      "lambda 1e-2, held-out seeds",
            "plain_ms": float(np.median([r["plain_ms"] for r in rows])),
            "learned_ms": float(np.median([r["learned_ms"] for r in rows])),
            "learned_faster": int(sum(r["learned_ms"] < r["plain_ms"] for r in rows)),
            "seeds": len(rows), "problems": rows}


def batched_cor1(tomo, ts, iters=10, reps=3):
    """COR1-like batch: 8 time frames of 256^3 on [-4, 4]^3 (60 views of
    512x512, detector annulus 1.4-4 kept, unit sphere masked, temporal prior
    lambda_t 10) plus 4 independent reconstructions of 64^3-192^3 (16 views
    of 256x256 each), every launch shape chosen by the autotuner for its size
    class.  Times `iters` CG iterations of all five systems in the batched
    persistent launches with graph-captured check intervals (median of
    `reps`) against the same iterations run system after system."""
    import torch

    wl = ts.cor1_frames()
    extras = ts.cor1_extras()
    works = [wl] + extras
    dgs = [tomo.DeviceGeometry(w.geom) for w in works]
    tunings = [tomo.autotune(dg, reps=2) for dg in dgs]
    ys = [tomo.project(dg, torch.as_tensor(w.x.astype(np.float32)).cuda()) for dg, w in zip(dgs, works)]
    cross = [tomo.count_crossings(dg) for dg in dgs]
    lam_t = [w.lam_t for w in works]
    batch = tomo.Batch(dgs)

    def run_batch():
        return batch.cg_solve(ys, lam_r=1e-2, lam_t=lam_t, max_iter=iters, check_every=iters, use_graph=True)

    def run_seq():
        for dg, y, lt in zip(dgs, ys, lam_t):
            tomo.cg_solve(dg, y, lam_r=1e-2, lam_t=lt, max_iter=iters, check_every=iters)

    def timed(f):
        f()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            t0 = time.perf_counter()
            f()
            torch.cuda.synchronize()
            out.append(time.perf_counter() - t0)
        return float(np.median(out))

    t_batch, t_seq = timed(run_batch), timed(run_seq)
    _, reps_b = run_batch()
    apps = sum(r["n_project"] + r["n_backproject"] for r in reps_b)
    per_app = {k: c for k, c in zip(range(len(cross)), cross)}
    crossings = sum((r["n_project"] + r["n_backproject"]) * per_app[k] for k, r in enumerate(reps_b))
    out = {"workload": "COR1-like: 8 frames of 256^3 (60 views of 512^2, annulus mask, lambda_t 10) + "
                       "64^3, 96^3, 128^3, 192^3 extras (16 views of 256^2), one persistent P and P^T "
                       "launch per operator, graph-captured CG",
           "iterations": iters, "systems": len(dgs), "applications": apps,
           "ms_batched": 1e3 * t_batch, "ms_sequential": 1e3 * t_seq, "speedup": t_seq / t_batch,
           "crossings_per_s": crossings / t_batch,
           "p_items": batch.items(0), "pt_items": batch.items(1), "p_workgroups": batch.items(2),
           "pt_workgroups": batch.items(3),
           "tuning": [{k: (list(v) if isinstance(v, tuple) else v) for k, v in t.items()} for t in tunings]}
    batch.close()
    tomo.autotune_clear()
    return out


def obstacle_euvi(tomo, ts, wl, y, reps=10):
    """The obstacle variant on the EUVI-like workload: the same views and
    cube with the photosphere (unit sphere at the centre) ending every line
    of sight.  P and P^T per launch (HIP events on the launch stream, median
    of `reps`) and one 50-iteration CG step."""
    import torch

    g0 = wl.geom
    g = ts.Geometry(g0.n, g0.lo, g0.hi, g0.views, g0.npix, map_mask=g0.map_mask,
                    obstacle=np.array([0.0, 0.0, 0.0, 1.0]))
    dg = tomo.DeviceGeometry(g)
    cross = tomo.count_crossings(dg)
    x = torch.zeros(dg.cube_shape, dtype=torch.float32, device="cuda")
    img = torch.empty_like(y)

    def per_launch(f):
        f()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            f()
            e1.record()
            e1.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(np.median(out))

    ms_p = per_launch(lambda: tomo.project(dg, x, out=img))
    ms_bp = per_launch(lambda: tomo.backproject(dg, y, out=x))
    tomo.cg_solve(dg, y, lam_r=wl.lam_r, max_iter=wl.cg_iters, out=x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep = tomo.cg_solve(dg, y, lam_r=wl.lam_r, max_iter=wl.cg_iters, out=x)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    apps = rep["n_project"] + rep["n_backproject"]
    return {"workload": "EUVI-like (as the headline) with the photosphere as obstacle: lines of sight end "
                        "where they enter the unit sphere",
            "crossings_per_application": cross, "k_project_ms": ms_p, "k_backproject_ms": ms_bp,
            "project_crossings_per_s": cross / (ms_p * 1e-3), "backproject_crossings_per_s": cross / (ms_bp * 1e-3),
            "ms_per_step": 1e3 * dt, "crossings_per_s": apps * cross / dt, "final_rel_res": rep["rel_res"]}


def thomson_cor1(tomo, ts, reps=5):
    """Thomson-scattering operators on a static COR1-like frame: 256^3 on
    [-4, 4]^3 R_sun, all 60 views of 512^2 (annulus 1.4-4 R_sun kept, unit
    sphere masked), u = 0.63: T_pB and T_B and their transposes per call
    (HIP events on the launch stream, median of `reps`)."""
    import torch

    wl = ts.cor1_frames(K=1)
    dg = tomo.DeviceGeometry(wl.geom)
    cross = tomo.count_crossings(dg)
    ne = torch.as_tensor(wl.x.reshape(dg.cube_shape).astype(np.float32)).cuda()
    img = torch.empty(dg.npix, dtype=torch.float32, device="cuda")
    back = torch.empty(dg.cube_shape, dtype=torch.float32, device="cuda")

    def per_call(f):
        f()
        torch.cuda.synchronize()
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            f()
            e1.record()
            e1.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(np.median(out))

    res = {"workload": "COR1-like static frame: 256^3 on [-4,4]^3 R_sun, 60 views of 512^2, annulus "
                       "1.4-4 R_sun, unit sphere masked, u 0.63",
           "crossings_per_projection": cross}
    for kind in ("pB", "B"):
        nproj = 1 if kind == "pB" else 2
        ms_f = per_call(lambda: tomo.thomson_project(dg, ne, 0.63, kind, out=img))
        ms_b = per_call(lambda: tomo.thomson_backproject(dg, img, 0.63, kind, out=back))
        res[kind] = {"project_ms": ms_f, "backproject_ms": ms_b,
                     "project_crossings_per_s": nproj * cross / (ms_f * 1e-3),
                     "backproject_crossings_per_s": nproj * cross / (ms_b * 1e-3)}
    return res


def height_gain_euvi(tomo, ts, wl, y, reps=10):
    """The multi-spacecraft inversion with the height-weighted prior on the
    EUVI-like workload: observer A's 14 views and observer B's 14 views as
    two instruments with gains 1 and 1.27 (B's data scaled to match), prior
    lambda R D^T D R with R the distance from the Sun's centre.  P and P^T
    with gains and the weighted prior per launch (HIP events on the launch
    stream, median of `reps`) next to the plain ones, and one 50-iteration
    CG step."""
    import torch

    g0 = wl.geom
    gains = np.where(np.arange(g0.nviews) % 2 == 1, 1.27, 1.0)
    g = ts.Geometry(g0.n, g0.lo, g0.hi, g0.views, g0.npix, map_mask=g0.map_mask, gains=gains)
    dg, d0 = tomo.DeviceGeometry(g), tomo.DeviceGeometry(g0)
    cross = tomo.count_crossings(dg)
    ray_gain = torch.as_tensor(np.repeat(gains, g0.npix[:, 0] * g0.npix[:, 1]).astype(np.float32)).cuda()
    y_ab = y * ray_gain
    height = (0.0, 0.0, 0.0, 0.0)
    x = torch.as_tensor(wl.x.astype(np.float32)).cuda()
    out = torch.empty_like(x)
    img = torch.empty_like(y)

    def per_launch(f):
        f()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            f()
            e1.record()
            e1.synchronize()
            t.append(e0.elapsed_time(e1))
        return float(np.median(t))

    ms = {"project_gains": per_launch(lambda: tomo.project(dg, x, out=img)),
          "project_plain": per_launch(lambda: tomo.project(d0, x, out=img)),
          "backproject_gains": per_launch(lambda: tomo.backproject(dg, y_ab, out=out)),
          "backproject_plain": per_launch(lambda: tomo.backproject(d0, y, out=out)),
          "prior_height": per_launch(lambda: tomo.apply_prior(dg, x, wl.lam_r, out=out, height=height)),
          "prior_plain": per_launch(lambda: tomo.apply_prior(dg, x, wl.lam_r, out=out))}
    vox = int(np.prod(g0.n))
    tomo.cg_solve(dg, y_ab, lam_r=wl.lam_r, max_iter=wl.cg_iters, out=out, height=height)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep = tomo.cg_solve(dg, y_ab, lam_r=wl.lam_r, max_iter=wl.cg_iters, out=out, height=height)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    apps = rep["n_project"] + rep["n_backproject"]
    return {"workload": "EUVI-like (as the headline) as two instruments, observer B at gain 1.27, "
                        "height-weighted prior (R = distance from the Sun's centre), lambda 1e-2",
            "crossings_per_application": cross,
            "kernel_ms": ms,
            "prior_height_gbs": 8.0 * vox / (ms["prior_height"] * 1e-3) / 1e9,
            "ms_per_step": 1e3 * dt, "crossings_per_s": apps * cross / dt, "final_rel_res": rep["rel_res"]}


# The paper's projector timings (Sec. "Performance", image-size and cube-size
# tables; 64 images, no mask, no obstacle; two quad-core Opteron 2380), in
# seconds per projection and back-projection, for context only.
PAPER_IMAGE_S = {128: (0.95, 1.61), 256: (3.64, 6.17), 512: (14.53, 24.69), 1024: (58.75, 99.54)}
PAPER_CUBE_S = {128: (13.84, 24.71), 256: (44.56, 56.64), 512: (195.69, 214.55), 1024: (587.56, 610.75)}


def sweeps(tomo, ts, reps=5, only=None, tune=True):
    """The paper's projector scaling sweeps on the GPU: 64 views, no mask,
    no obstacle; image sides 128..1024 on a 128^3 cube, then cube sides
    128..1024 (up to 2^30 voxels, 4 GiB) under 256^2 images.  Per point:
    crossings, P and blocked P^T per launch with the default launch shapes
    and after tomo_autotune on the point (HIP events on the launch stream,
    median of `reps`), crossings/s and algorithmic GB/s of the tuned launches
    (4 B per crossing + 4 B per ray for P, 8 B + 4 B for P^T), and the
    paper's seconds.  only = (cube side, image side) runs that single point;
    tune = False keeps the default shapes (for profiling one shape)."""
    import torch

    def per_launch(f):
        f()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            f()
            e1.record()
            e1.synchronize()
            t.append(e0.elapsed_time(e1))
        return float(np.median(t))

    def point(n, npix, paper):
        g = ts.sweep_geometry(n, npix)
        dg = tomo.DeviceGeometry(g)
        x = torch.as_tensor(ts.sweep_cube(ts.sweep_cube_parts(n))).cuda()
        tomo.autotune_clear()  # the default shapes, whatever an earlier point of this class tuned
        y = tomo.project(dg, x)
        out = torch.empty_like(x)
        cross = tomo.count_crossings(dg)
        ms_p0 = per_launch(lambda: tomo.project(dg, x, out=y))
        ms_b0 = per_launch(lambda: tomo.backproject(dg, y, out=out, strategy=tomo.BP_BLOCKED))
        tuned, t_tune, ms_p, ms_b = None, 0.0, ms_p0, ms_b0
        if tune:
            t0 = time.perf_counter()
            tuned = tomo.autotune(dg, reps=5)
            t_tune = time.perf_counter() - t0
            ms_p = per_launch(lambda: tomo.project(dg, x, out=y))
            ms_b = per_launch(lambda: tomo.backproject(dg, y, out=out))
        rays = g.nrays
        res = {"cube": n, "image": npix, "rays": rays, "crossings": cross,
               "default_project_ms": ms_p0, "default_backproject_ms": ms_b0,
               "project_ms": ms_p, "backproject_ms": ms_b, "tuning": tuned, "autotune_s": t_tune,
               "project_crossings_per_s": cross / (ms_p * 1e-3),
               "backproject_crossings_per_s": cross / (ms_b * 1e-3),
               "project_gbs": (4.0 * cross + 4.0 * rays) / (ms_p * 1e-3) / 1e9,
               "backproject_gbs": (8.0 * cross + 4.0 * rays) / (ms_b * 1e-3) / 1e9,
               "paper_project_s": paper[0], "paper_backproject_s": paper[1]}
        del x, y, out, dg
        torch.cuda.empty_cache()
        return res

    if only is not None:
        n, npix = only
        paper = PAPER_CUBE_S.get(n) if npix == 256 else PAPER_IMAGE_S.get(npix) if n == 128 else None
        image, cube = [], [point(n, npix, paper or (None, None))]
    else:
        image = [point(128, s, PAPER_IMAGE_S[s]) for s in ts.SWEEP_IMAGE_SIDES]
        log("image-size sweep done")
        cube = [point(s, 256, PAPER_CUBE_S[s]) for s in ts.SWEEP_CUBE_SIDES]
        log("cube-size sweep done")
    tomo.autotune_clear()
    return {"workload": "the paper's projector benchmark: 64 views at 215 R_sun around the equator, FOV 3.2, "
                        "cube on [-1.5,1.5]^3, no mask, no obstacle; paper times for context (other hardware)",
            "image_size": image, "cube_size": cube}


def per_config(tomo, ts, reps=20):
    """P and the default P^T per launch on the other configurations' geometries
    (HIP events on the launch stream, median of `reps` after 3 warm-ups):
    the tiny 32^3 problem, one COR1-like 256^3 frame with its masks, the
    differentiable 128^3 / 32 x 256^2 set-up and a learned-preconditioner
    problem (128^3, 28 x 256^2)."""
    import torch

    def per_launch(f):
        for _ in range(3):
            f()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            f()
            e1.record()
            e1.synchronize()
            t.append(e0.elapsed_time(e1))
        return float(np.median(t))

    out = {}
    for name, wl in (("tiny", ts.tiny()), ("cor1_frame", ts.cor1_frames(K=1)),
                     ("differentiable", ts.differentiable()), ("learned", ts.learned(2003))):
        dg = tomo.DeviceGeometry(wl.geom)
        x = torch.as_tensor(wl.x.reshape(dg.cube_shape).astype(np.float32)).cuda()
        y = tomo.project(dg, x)
        back = torch.empty_like(x)
        cross = tomo.count_crossings(dg)
        ms_p = per_launch(lambda: tomo.project(dg, x, out=y))
        ms_b = per_launch(lambda: tomo.backproject(dg, y, out=back))
        out[name] = {"geometry": wl.name, "crossings": cross, "project_ms": ms_p, "backproject_ms": ms_b,
                     "project_crossings_per_s": cross / (ms_p * 1e-3),
                     "backproject_crossings_per_s": cross / (ms_b * 1e-3)}
        del dg, x, y, back
        torch.cuda.empty_cache()
    return out


def cpu_baseline(wl, reps, ts_mod):
    """The FP64 oracle (as it stands) on a bounded sample: `reps` passes of
    P and P^T over the full geometry (the CG's operator pair), all host
    cores."""
    import oracle as ora

    g = wl.geom
    cross = ora.count_crossings(g)
    y = np.random.default_rng(0).normal(size=g.nrays)
    t0 = time.perf_counter()
    for _ in range(reps):
        ora.project(g, wl.x)
        ora.backproject(g, y)
    dt = time.perf_counter() - t0
    cores = ora.max_threads()
    # one host thread on a smaller sample: two of the views, one pass (the
    # oracle's thread count persists, so it is set back afterwards)
    g2 = g.subset([0, 1])
    c2 = ora.count_crossings(g2)
    y2 = y[:g2.nrays]
    t1 = time.perf_counter()
    ora.project(g2, wl.x, nthreads=1)
    ora.backproject(g2, y2, nthreads=1)
    dt1 = time.perf_counter() - t1
    ora.count_crossings(g2, nthreads=cores)
    # the other configurations, one P + P^T pass each on all cores (one
    # COR1-like frame for the batched configuration)
    others = {}
    for name, w2 in (("tiny", ts_mod.tiny()), ("differentiable", ts_mod.differentiable()),
                     ("learned", ts_mod.learned(2003)), ("cor1_frame", ts_mod.cor1_frames(K=1))):
        gg = w2.geom
        cc = ora.count_crossings(gg)
        yy = np.random.default_rng(1).normal(size=gg.nrays)
        t2 = time.perf_counter()
        ora.project(gg, w2.x)
        ora.backproject(gg, yy)
        others[name] = {"crossings_per_s": 2.0 * cc / (time.perf_counter() - t2), "crossings": cc}
    return {"value": 2.0 * reps * cross / dt, "unit": "voxel-crossings/s",
            "cores": cores, "kind": "oracle",
            "sample": f"{reps} x (P + P^T) over all 28 views of 512x512 and the 128^3 EUVI-like "
                      f"cube ({cross} crossings per application), {dt:.1f} s",
            "one_thread": {"value": 2.0 * c2 / dt1, "cores": 1,
                           "sample": f"1 x (P + P^T) over 2 of the views ({c2} crossings), {dt1:.1f} s"},
            "other_configs": others}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU (--gpus 1); the "
                                   "library has no multi-GPU path"}))
        sys.exit(2)
    import torch

    import paper_1103_5904_amd as tomo
    import tomo_synth as ts

    torch.cuda.set_device(0)
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.sweep_only is not None:
        print(json.dumps({"sweep": sweeps(tomo, ts, only=tuple(args.sweep_only),
                                          tune=not args.sweep_no_autotune)}), flush=True)
        return
    wl = ts.euvi()
    g = wl.geom
    dg = tomo.DeviceGeometry(g)
    x_true = torch.as_tensor(wl.x.astype(np.float32)).cuda()
    y = tomo.project(dg, x_true)
    rms = float(torch.sqrt(torch.mean(y.double() ** 2)))
    y += torch.as_tensor(ts.gaussian_noise(g.nrays, wl.noise_rel * rms, wl.noise_seed)
                         .astype(np.float32)).cuda()
    crossings = tomo.count_crossings(dg)
    x = torch.empty(dg.cube_shape, dtype=torch.float32, device="cuda")

    bp = {"auto": tomo.BP_AUTO, "binned": tomo.BP_BINNED, "atomic": tomo.BP_ATOMIC,
          "blocked": tomo.BP_BLOCKED}[args.bp]

    def step():
        return tomo.cg_solve(dg, y, lam_r=wl.lam_r, max_iter=wl.cg_iters, time_kernels=True, out=x,
                             bp_strategy=bp)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        reps.append(step()[1])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    apps = sum(r["n_project"] + r["n_backproject"] for r in reps) / args.steps
    value = apps * crossings / (ms_step * 1e-3)

    # per-launch kernel times (events around each P and P^T inside the solve)
    n_it = sum(r["iters"] for r in reps)
    ms_p = sum(r["ms_project"] for r in reps) / n_it
    ms_bp = sum(r["ms_backproject"] for r in reps) / n_it
    nrays = dg.npix
    bytes_p = 4.0 * crossings + 4.0 * nrays
    bytes_bp = 8.0 * crossings + 4.0 * nrays
    bp_used = args.bp if args.bp != "auto" else \
        {1: "atomic", 2: "binned", 3: "blocked"}[tomo.get_tuning()["bp_default"]]
    if ms_bp >= ms_p:
        dom = f"k_backproject_{bp_used}"
        ms_dom, b_dom = ms_bp, bytes_bp
    else:
        dom, ms_dom, b_dom = "k_project", ms_p, bytes_p
    achieved = b_dom / (ms_dom * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-crossings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "EUVI-like static inversion: 128^3 cube on [-1.5,1.5]^3 R_sun, "
                               "unit sphere masked, 28 views of 512x512 at FOV 3.4, 50 CG "
                               "iterations, lambda 1e-2",
                   "crossings_per_application": crossings, "applications_per_step": apps,
                   "rays": nrays, "storage": "f32", "walk": "f64",
                   "final_rel_res": reps[-1]["rel_res"], "backprojection": bp_used},
        "kernels": {"k_project_ms": ms_p, "k_backproject_ms": ms_bp,
                    "project_crossings_per_s": crossings / (ms_p * 1e-3),
                    "backproject_crossings_per_s": crossings / (ms_bp * 1e-3)},
        "roofline": {"kernel": dom, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom)},
    }
    gbs_p, gbs_bp = bytes_p / (ms_p * 1e-3) / 1e9, bytes_bp / (ms_bp * 1e-3) / 1e9
    pr = probes() if not args.no_probes else None
    if pr:
        out["achievable"] = {**pr,
                             "project_gbs": gbs_p, "backproject_gbs": gbs_bp,
                             "project_frac_hbm": gbs_p / pr["hbm_copy_gbs"],
                             "project_frac_mall": gbs_p / pr["mall_copy_gbs"],
                             "backproject_frac_hbm": gbs_bp / pr["hbm_copy_gbs"],
                             "backproject_frac_mall": gbs_bp / pr["mall_copy_gbs"]}
    ceil_p = VALU_LANE_RATE / VALU_PER_CROSSING["k_project"]
    ceil_bp = VALU_LANE_RATE / VALU_PER_CROSSING["k_backproject_blocked"]
    out["valu"] = {"instr_per_crossing": VALU_PER_CROSSING,
                   "project_ceiling_crossings_per_s": ceil_p,
                   "project_frac": crossings / (ms_p * 1e-3) / ceil_p,
                   "backproject_ceiling_crossings_per_s": ceil_bp,
                   "backproject_frac": crossings / (ms_bp * 1e-3) / ceil_bp}
    log(f"timed steps done: {ms_step:.1f} ms per step")
    if not args.no_learned:
        out["time_to_rel_res_1e-3"] = learned_vs_plain(tomo, ts)
        log("learned vs plain done")
    if not args.no_batch:
        out["batched"] = batched_cor1(tomo, ts)
        log("batched COR1-like done")
    if not args.no_obstacle:
        out["obstacle"] = obstacle_euvi(tomo, ts, wl, y)
        log("obstacle variant done")
    if not args.no_thomson:
        out["thomson"] = thomson_cor1(tomo, ts)
        log("Thomson operators done")
    if not args.no_height_gain:
        out["height_gain"] = height_gain_euvi(tomo, ts, wl, y)
        log("two instruments with the height-weighted prior done")
    if not args.no_configs:
        out["configs"] = per_config(tomo, ts)
        log("per-configuration P and P^T done")
    if not args.no_sweep:
        out["sweep"] = sweeps(tomo, ts, tune=not args.sweep_no_autotune)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_reps, ts)
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
