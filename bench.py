"""Benchmark: Siddon P / P^T voxel-crossings per second on one MI355X.

One step is the COR1-like batched time-evolving inversion, the largest
configuration that fits one GPU: 8 time-frame cubes of 256^3 on [-4, 4]^3
R_sun (60 views of 512x512, detector annulus 1.4-4 R_sun kept, unit sphere
masked, temporal prior lambda_t 10) plus four independent reconstructions of
64^3, 96^3, 128^3 and 192^3 (16 views of 256x256 each), solved together by
the batched CG: per iteration each system's own P launch and one persistent
P^T launch over all five systems, each check interval replayed from a HIP
graph, launch shapes chosen by the autotuner per size class.  A step is one
such solve of --iters iterations (one P^T for the right-hand side, per
iteration one P and one P^T, one P and P^T for the final true residual).
Inputs are synthetic, generated once and resident in HBM before timing.

value = (P and P^T applications in the step, per system) x (voxel crossings
per application of that system) / step time.  The roofline entry is for the
batched kernel that takes most of the step, its per-launch time from HIP
events the library records around every batched launch on the launch
stream (as graph nodes) during the timed steps.  The kernels are bound by
vector-ALU issue, not by memory: the roofline reports issued VALU lane-
instructions per second (the profiled instruction count of one launch over
its live duration) against 256 CUs x 64 lanes x 2.4 GHz, with the
algorithmic and the measured HBM bytes beside it.

Secondary figures, each a short summary on the line (full tables in the
details file, --details): the same batch solved system after system
(batched), the EUVI-like static inversion (euvi), learned flexible CG
against plain CG to relative residual 1e-3 on held-out problems
(time_to_rel_res_1e-3), the obstacle variant (obstacle), the Thomson
operators (thomson), two instruments with the height-weighted prior
(height_gain), P and P^T on the other configurations (configs), the paper's
projector scaling sweeps (sweep), and the FP64 oracle on the host's cores
(cpu_baseline).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Siddon P/Pᵀ voxel-crossings/s; time to rel. residual 1e-3 (learned vs plain)"
HBM_PEAK_GBS = 8000.0
# VALU issue ceiling: 256 CUs, each issuing 64 lanes of vector instructions per
# clock (four SIMDs, one wave64 instruction every four clocks each; FP64 at
# the full rate on gfx950), at 2.4 GHz.  In flops this is the FP64 vector
# peak, 78.6 TFLOP/s, with an FMA counted as two.
VALU_PEAK_LANE_INSTR = 256 * 64 * 2.4e9
# VALU instructions of one voxel crossing in the walk loop of each kernel of
# an iteration (its four-crossing loop body in the gfx950 ISA, divided by
# four): the P^T walk with its fixed-point LDS deposit at the bin's LDS
# address (batch.hip; 88 VALU per loop body), and the
# P gather-FMA walk over the 16^3-bricked cube of the dominant system with
# its offsets from the LDS table of per-axis terms (siddon.hip; 106 VALU per
# loop body, six of them register moves at the loop's back edge).
WALK_VALU_PER_CROSSING = {"k_project_bricked_lut": 106 / 4, "k_batch_backproject": 88 / 4}

# Per-launch counters of the batched kernels on the headline step, from
# rocprofv3 --pmc passes of `bench.py --headline-only` (profiles/
# cor1_batch_backprojection.md): SQ_INSTS_VALU (wave-level VALU instructions
# per dispatch) and the HBM bytes per dispatch (FETCH_SIZE x 1.9997 +
# WRITE_SIZE, the scale factors a 256 MiB device copy reads).  Valid only for
# the sources they were taken on: sha256 over the listed files, first 16 hex
# digits; otherwise the fields they feed are null.
PROFILED = {
    "k_batch_backproject": {"sha": "e45dfa706beb9e49", "valu_insts": 2633252128.0, "hbm_bytes": 9116604475.5},
}
PROFILED_FILES = ["blocked.h", "batch.hip", "batch.h", "walk.h", "common.h", "api.hip", "tune.hip"]


def sources_digest(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1103_5904_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled(kernel):
    ent = PROFILED.get(kernel)
    if ent is None or ent.get("sha") != sources_digest(PROFILED_FILES):
        return None
    return ent


def log(msg):
    """Progress on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=50, help="CG iterations per step")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed headline steps (for profiling them)")
    ap.add_argument("--no-autotune", action="store_true", help="headline with the default launch shapes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=3, help="timed oracle passes (median), after one warm-up")
    for part in ("sequential", "euvi", "learned", "obstacle", "thomson", "height-gain", "configs", "sweep",
                 "probes"):
        ap.add_argument(f"--no-{part}", action="store_true", help=f"skip the {part} figures")
    ap.add_argument("--sweep-only", type=int, nargs=2, metavar=("CUBE", "IMAGE"), default=None,
                    help="run only the sweep point with this cube side and image side, and print its line")
    ap.add_argument("--sweep-no-autotune", action="store_true",
                    help="time the sweep with the default launch shapes only")
    ap.add_argument("--euvi-only", action="store_true", help="only the EUVI-like step (for profiling it)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="before anything else, run 3 device-to-device copies of MIB MiB: the known-size "
                         "kernel that calibrates hardware byte counters")
    ap.add_argument("--details", default=os.path.join(ROOT, "gpurun_out", "bench_details.json"),
                    help="file for the full per-seed, per-point and per-configuration tables")
    return ap.parse_args()


def events_ms(f, reps, warm=3):
    """Median wall time of f() between HIP events on the current stream (the
    stream the library launches on), after `warm` untimed calls."""
    import torch

    for _ in range(warm):
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


def probes(reps=5):
    """Achievable bandwidths measured with plain device copies (torch): a
    2 GiB buffer (HBM) and a 32 MiB buffer copied 20 times over (resident in
    the 256 MB Infinity Cache).  Bytes read + written per second, median of
    `reps`."""
    import torch

    def rate(nbytes, inner):
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)

        def f():
            for _ in range(inner):
                dst.copy_(src)

        ms = events_ms(f, reps, warm=1)
        del src, dst
        torch.cuda.empty_cache()
        return 2.0 * nbytes * inner / (ms * 1e-3) / 1e9

    return {"hbm_copy_gbs": rate(2 << 30, 1), "mall_copy_gbs": rate(32 << 20, 20)}


# ------------------------------------------------------------------ headline


class Cor1Batch:
    """The COR1-like batch on the device: geometries, data, crossing counts."""

    def __init__(self, tomo, ts, autotune=True):
        import torch

        self.works = [ts.cor1_frames()] + ts.cor1_extras()
        self.dgs = [tomo.DeviceGeometry(w.geom) for w in self.works]
        self.tunings = [tomo.autotune(dg, reps=3) for dg in self.dgs] if autotune else None
        self.xs = [torch.as_tensor(w.x.astype(np.float32)).cuda() for w in self.works]
        self.ys = [tomo.project(dg, x) for dg, x in zip(self.dgs, self.xs)]
        self.cross = [tomo.count_crossings(dg) for dg in self.dgs]
        self.rays = [dg.npix for dg in self.dgs]
        self.lam_t = [w.lam_t for w in self.works]
        self.batch = tomo.Batch(self.dgs)

    def solve(self, iters, time_kernels=True):
        return self.batch.cg_solve(self.ys, lam_r=1e-2, lam_t=self.lam_t, max_iter=iters, check_every=iters,
                                   use_graph=True, time_kernels=time_kernels)

    def crossings_of(self, reps):
        return sum((r["n_project"] + r["n_backproject"]) * c for r, c in zip(reps, self.cross))


def headline(tomo, ts, args):
    import torch

    log("COR1-like batch: set-up and autotuning")
    cb = Cor1Batch(tomo, ts, autotune=not args.no_autotune)
    for _ in range(args.warmup):
        cb.solve(args.iters)
    torch.cuda.synchronize()
    reps_all = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        reps_all.append(cb.solve(args.iters)[1])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_step = 1e3 * dt / args.steps
    crossings = sum(cb.crossings_of(r) for r in reps_all) / args.steps
    apps = sum(r["n_project"] + r["n_backproject"] for r in reps_all[0])
    log(f"timed steps done: {ms_step:.1f} ms per step")
    # per-launch times of the batched kernels during the timed steps
    launches = args.steps * max(r["iters"] for r in reps_all[0])
    ms_p = sum(rr[0]["ms_project"] for rr in reps_all) / launches
    ms_b = sum(rr[0]["ms_backproject"] for rr in reps_all) / launches
    xp, xb = sum(cb.cross), sum(cb.cross)  # every system applies each operator once per launch
    rays = sum(cb.rays)
    return cb, {"ms_step": ms_step, "value": crossings / (ms_step * 1e-3), "applications": apps,
                "ms_p": ms_p, "ms_b": ms_b, "cross_p": xp, "cross_b": xb, "rays": rays,
                "final_rel_res": [r["rel_res"] for r in reps_all[-1]]}


def roofline(h):
    """The dominant batched kernel against the VALU issue ceiling.

    achieved = (walk-loop VALU lane-instructions per voxel crossing, counted
    in the kernel's gfx950 ISA) x (crossings of one launch) / (the launch's
    live duration): the walk's own arithmetic, the algorithmic unit of this
    bound.  issued_frac counts every VALU instruction the launch issued
    (ray set-ups, footprints, idle lanes of diverged wavefronts included),
    from the profiled SQ_INSTS_VALU; traffic is the profiled HBM bytes of one
    launch.  Both are null when the sources changed since they were taken."""
    if h["ms_b"] >= h["ms_p"]:
        kern, ms, cross = "k_batch_backproject", h["ms_b"], h["cross_b"]
        alg = 8.0 * cross + 4.0 * h["rays"]
    else:
        kern, ms, cross = "k_project_bricked_lut", h["ms_p"], h["cross_p"]
        alg = 4.0 * cross + 4.0 * h["rays"]
    sec = ms * 1e-3
    per = WALK_VALU_PER_CROSSING[kern]
    peak = VALU_PEAK_LANE_INSTR / 1e12
    achieved = per * cross / sec / 1e12
    out = {"kernel": kern, "bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tinstr/s",
           "frac": achieved / peak, "traffic": None, "launch_ms": ms, "valu_per_crossing": per,
           "algorithmic_bytes": alg, "algorithmic_frac_hbm": alg / sec / 1e9 / HBM_PEAK_GBS}
    prof = profiled(kern)
    if prof is not None:
        issued = prof["valu_insts"] * 64.0 / sec / 1e12
        out.update({"issued_frac": issued / peak, "traffic": prof["hbm_bytes"],
                    "traffic_over_algorithmic": prof["hbm_bytes"] / alg})
    else:
        out.update({"issued_frac": None, "note": "kernel sources changed since the counters were profiled"})
    return out


def sequential(tomo, cb, iters, reps=3):
    """The same CG iterations run system after system (tomo_cg_solve each,
    blocked P^T, the same tunings), median of `reps` after one warm-up."""
    import torch

    def run():
        for dg, y, lt in zip(cb.dgs, cb.ys, cb.lam_t):
            tomo.cg_solve(dg, y, lam_r=1e-2, lam_t=lt, max_iter=iters, check_every=iters,
                          bp_strategy=tomo.BP_BLOCKED)

    run()
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        t.append(time.perf_counter() - t0)
    return 1e3 * float(np.median(t))


# --------------------------------------------------------- secondary figures


def euvi_step(tomo, ts, steps=5):
    """The EUVI-like static inversion: 50 CG iterations on the 128^3 cube
    (unit sphere masked) seen by 28 views of 512x512 with 1% noise; P and
    P^T per launch from events inside the solve."""
    import torch

    wl = ts.euvi()
    dg = tomo.DeviceGeometry(wl.geom)
    y = tomo.project(dg, torch.as_tensor(wl.x.astype(np.float32)).cuda())
    rms = float(torch.sqrt(torch.mean(y.double() ** 2)))
    y += torch.as_tensor(ts.gaussian_noise(wl.geom.nrays, wl.noise_rel * rms, wl.noise_seed)
                         .astype(np.float32)).cuda()
    cross = tomo.count_crossings(dg)
    x = torch.empty(dg.cube_shape, dtype=torch.float32, device="cuda")

    def step():
        return tomo.cg_solve(dg, y, lam_r=wl.lam_r, max_iter=wl.cg_iters, time_kernels=True, out=x)[1]

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    n_it = sum(r["iters"] for r in reps)
    ms_p = sum(r["ms_project"] for r in reps) / n_it
    ms_b = sum(r["ms_backproject"] for r in reps) / n_it
    apps = reps[0]["n_project"] + reps[0]["n_backproject"]
    return wl, dg, y, {"ms_per_step": 1e3 * dt, "crossings_per_s": apps * cross / dt,
                       "crossings_per_application": cross, "k_project_ms": ms_p, "k_backproject_ms": ms_b,
                       "project_crossings_per_s": cross / (ms_p * 1e-3),
                       "backproject_crossings_per_s": cross / (ms_b * 1e-3)}


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
        y = pc.noisy_data(dg, torch.as_tensor(wl.x.astype(np.float32)).cuda(), wl.noise_rel, wl.noise_seed)
        res = {"seed": seed}
        for name, params in (("plain", None), ("learned", net)):
            pc.time_to_tolerance(dg, y, wl.lam_r, 1e-3, params)
            ms, rep = pc.time_to_tolerance(dg, y, wl.lam_r, 1e-3, params, reps=reps)
            res[f"{name}_ms"] = ms
            res[f"{name}_iters"] = rep["iters"]
            res[f"{name}_true_rel_res"] = rep["true_rel_res"]
        res["speedup"] = res["plain_ms"] / res["learned_ms"]
        rows.append(res)
    plain = float(np.median([r["plain_ms"] for r in rows]))
    learned = float(np.median([r["learned_ms"] for r in rows]))
    summary = {"plain_ms": plain, "learned_ms": learned, "speedup": plain / learned,
               "learned_faster": int(sum(r["learned_ms"] < r["plain_ms"] for r in rows)), "seeds": len(rows),
               "min_speedup": float(min(r["speedup"] for r in rows)),
               "plain_iters": float(np.median([r["plain_iters"] for r in rows])),
               "learned_iters": float(np.median([r["learned_iters"] for r in rows]))}
    return summary, {"rtol": 1e-3, "workload": "128^3 blob phantom, 28 views of 256x256, 1% noise, lambda 1e-2, "
                                               "held-out seeds", "problems": rows}


def obstacle_euvi(tomo, ts, wl, y, reps=10):
    """The obstacle variant on the EUVI-like workload: lines of sight end
    where they enter the unit sphere.  One 50-iteration CG step, with P and
    P^T per launch from events inside the solve (as for the EUVI-like step),
    and the standalone tomo_backproject call beside them (no ray table)."""
    import torch

    g0 = wl.geom
    g = ts.Geometry(g0.n, g0.lo, g0.hi, g0.views, g0.npix, map_mask=g0.map_mask,
                    obstacle=np.array([0.0, 0.0, 0.0, 1.0]))
    dg = tomo.DeviceGeometry(g)
    cross = tomo.count_crossings(dg)
    x = torch.zeros(dg.cube_shape, dtype=torch.float32, device="cuda")
    ms_call = events_ms(lambda: tomo.backproject(dg, y, out=x), reps)
    tomo.cg_solve(dg, y, lam_r=wl.lam_r, max_iter=wl.cg_iters, out=x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rep = tomo.cg_solve(dg, y, lam_r=wl.lam_r, max_iter=wl.cg_iters, out=x, time_kernels=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"crossings": cross, "k_project_ms": rep["ms_project"] / rep["n_project"],
            "k_backproject_ms": rep["ms_backproject"] / rep["n_backproject"], "backproject_call_ms": ms_call,
            "ms_per_step": 1e3 * dt, "crossings_per_s": (rep["n_project"] + rep["n_backproject"]) * cross / dt}


def thomson_cor1(tomo, ts, reps=5):
    """T_pB and T_B and their transposes per call on a static COR1-like
    frame (256^3, 60 views of 512^2, annulus kept, unit sphere masked,
    u = 0.63): ms forward, ms transpose."""
    import torch

    wl = ts.cor1_frames(K=1)
    dg = tomo.DeviceGeometry(wl.geom)
    ne = torch.as_tensor(wl.x.reshape(dg.cube_shape).astype(np.float32)).cuda()
    img = torch.empty(dg.npix, dtype=torch.float32, device="cuda")
    back = torch.empty(dg.cube_shape, dtype=torch.float32, device="cuda")
    out = {}
    for kind in ("pB", "B"):
        out[kind] = [events_ms(lambda: tomo.thomson_project(dg, ne, 0.63, kind, out=img), reps),
                     events_ms(lambda: tomo.thomson_backproject(dg, img, 0.63, kind, out=back), reps)]
    return out


def height_gain_euvi(tomo, ts, wl, y, reps=10):
    """The EUVI-like workload as two instruments (observer B at gain 1.27,
    its data scaled to match) with the height-weighted prior (R = distance
    from the Sun's centre): the prior kernels per launch and one 50-iteration
    CG step."""
    import torch

    g0 = wl.geom
    gains = np.where(np.arange(g0.nviews) % 2 == 1, 1.27, 1.0)
    g = ts.Geometry(g0.n, g0.lo, g0.hi, g0.views, g0.npix, map_mask=g0.map_mask, gains=gains)
    dg = tomo.DeviceGeometry(g)
    ray_gain = torch.as_tensor(np.repeat(gains, g0.npix[:, 0] * g0.npix[:, 1]).astype(np.float32)).cuda()
    y_ab = y * ray_gain
    height = (0.0, 0.0, 0.0, 0.0)
    x = torch.as_tensor(wl.x.astype(np.float32)).cuda()
    out = torch.empty_like(x)
    us_h = 1e3 * events_ms(lambda: tomo.apply_prior(dg, x, wl.lam_r, out=out, height=height), reps)
    us_p = 1e3 * events_ms(lambda: tomo.apply_prior(dg, x, wl.lam_r, out=out), reps)
    tomo.cg_solve(dg, y_ab, lam_r=wl.lam_r, max_iter=wl.cg_iters, out=out, height=height)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tomo.cg_solve(dg, y_ab, lam_r=wl.lam_r, max_iter=wl.cg_iters, out=out, height=height)
    torch.cuda.synchronize()
    return {"ms_per_step": 1e3 * (time.perf_counter() - t0), "prior_height_us": us_h, "prior_plain_us": us_p}


# The paper's projector timings (Sec. "Performance", image-size and cube-size
# tables; 64 images, no mask, no obstacle; two quad-core Opteron 2380), in
# seconds per projection and back-projection, for context only.
PAPER_IMAGE_S = {128: (0.95, 1.61), 256: (3.64, 6.17), 512: (14.53, 24.69), 1024: (58.75, 99.54)}
PAPER_CUBE_S = {128: (13.84, 24.71), 256: (44.56, 56.64), 512: (195.69, 214.55), 1024: (587.56, 610.75)}


def sweeps(tomo, ts, reps=5, only=None, tune=True):
    """The paper's projector scaling sweeps on the GPU: 64 views, no mask,
    no obstacle; image sides 128..1024 on a 128^3 cube, then cube sides
    128..1024 (up to 2^30 voxels, 4 GiB) under 256^2 images.  Per point:
    crossings, P and P^T per launch with the default launch shapes and after
    tomo_autotune on the point (median of `reps`), crossings/s and
    algorithmic GB/s of the tuned launches (4 B per crossing + 4 B per ray
    for P, 8 B + 4 B for P^T), and the paper's seconds."""
    import torch

    def point(n, npix, paper):
        g = ts.sweep_geometry(n, npix)
        dg = tomo.DeviceGeometry(g)
        x = torch.as_tensor(ts.sweep_cube(ts.sweep_cube_parts(n))).cuda()
        tomo.autotune_clear()  # the default shapes, whatever an earlier point of this class tuned
        y = tomo.project(dg, x)
        out = torch.empty_like(x)
        cross = tomo.count_crossings(dg)
        ms_p0 = events_ms(lambda: tomo.project(dg, x, out=y), reps)
        ms_b0 = events_ms(lambda: tomo.backproject(dg, y, out=out), reps)
        tuned, t_tune, ms_p, ms_b = None, 0.0, ms_p0, ms_b0
        if tune:
            t0 = time.perf_counter()
            tuned = tomo.autotune(dg, reps=5)
            t_tune = time.perf_counter() - t0
            ms_p = events_ms(lambda: tomo.project(dg, x, out=y), reps)
            ms_b = events_ms(lambda: tomo.backproject(dg, y, out=out), reps)
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
        pts = [point(n, npix, paper or (None, None))]
    else:
        pts = [point(128, s, PAPER_IMAGE_S[s]) for s in ts.SWEEP_IMAGE_SIDES]
        log("image-size sweep done")
        pts += [point(s, 256, PAPER_CUBE_S[s]) for s in ts.SWEEP_CUBE_SIDES]
        log("cube-size sweep done")
    tomo.autotune_clear()
    summary = [[p["cube"], p["image"], round(p["project_ms"], 3), round(p["backproject_ms"], 3),
                round(p["default_project_ms"], 3), round(p["default_backproject_ms"], 3)] for p in pts]
    return summary, {"workload": "the paper's projector benchmark: 64 views at 215 R_sun around the equator, "
                                 "FOV 3.2, cube on [-1.5,1.5]^3, no mask, no obstacle; paper times for context "
                                 "(other hardware)", "points": pts}


def per_config(tomo, ts, reps=20):
    """P and the default P^T per launch on the other configurations'
    geometries (median of `reps` after 3 warm-ups): the tiny 32^3 problem,
    one COR1-like 256^3 frame with its masks, the differentiable 128^3 / 32 x
    256^2 set-up and a learned-preconditioner problem (128^3, 28 x 256^2)."""
    import torch

    summary, details = {}, {}
    for name, wl in (("tiny", ts.tiny()), ("cor1_frame", ts.cor1_frames(K=1)),
                     ("differentiable", ts.differentiable()), ("learned", ts.learned(2003))):
        dg = tomo.DeviceGeometry(wl.geom)
        x = torch.as_tensor(wl.x.reshape(dg.cube_shape).astype(np.float32)).cuda()
        y = tomo.project(dg, x)
        back = torch.empty_like(x)
        cross = tomo.count_crossings(dg)
        ms_p = events_ms(lambda: tomo.project(dg, x, out=y), reps)
        ms_b = events_ms(lambda: tomo.backproject(dg, y, out=back), reps)
        summary[name] = [round(ms_p, 4), round(ms_b, 4)]
        details[name] = {"geometry": wl.name, "crossings": cross, "project_ms": ms_p, "backproject_ms": ms_b,
                         "project_crossings_per_s": cross / (ms_p * 1e-3),
                         "backproject_crossings_per_s": cross / (ms_b * 1e-3)}
        del dg, x, y, back
        torch.cuda.empty_cache()
    return summary, details


def cpu_baseline(ts_mod, reps):
    """The FP64 oracle (as it stands) on a bounded sample of the headline
    workload: P and P^T over the views of the first time frame of the
    COR1-like model (8 of its 60 views, that frame's 256^3 cube), all host
    cores, median of `reps` after one warm-up; and on one host thread, one
    of those views."""
    import oracle as ora

    wl = ts_mod.cor1_frames()
    g = wl.geom
    views0 = [int(v) for v in np.flatnonzero(g.view_frame == 0)]
    sub = g.subset(views0)
    cross = ora.count_crossings(sub)
    y = np.random.default_rng(0).normal(size=sub.nrays)

    def timed(geom, yy, nthreads):
        t0 = time.perf_counter()
        ora.project(geom, wl.x, nthreads=nthreads)
        ora.backproject(geom, yy, nthreads=nthreads)
        return time.perf_counter() - t0

    cores = ora.max_threads()
    timed(sub, y, 0)
    dt = float(np.median([timed(sub, y, 0) for _ in range(reps)]))
    one = sub.subset([0])
    c1 = ora.count_crossings(one)
    y1 = y[:one.nrays]
    timed(one, y1, 1)
    dt1 = float(np.median([timed(one, y1, 1) for _ in range(reps)]))
    ora.count_crossings(one, nthreads=cores)  # the oracle's thread count persists: restore it
    return {"value": 2.0 * cross / dt, "unit": "voxel-crossings/s", "cores": cores, "kind": "oracle",
            "sample": f"P + P^T over the {len(views0)} views of frame 0 of the COR1-like model (256^3, "
                      f"{cross} crossings per application), median of {reps} after one warm-up: {dt:.2f} s",
            "one_thread": {"value": 2.0 * c1 / dt1, "cores": 1,
                           "sample": f"P + P^T over 1 view ({c1} crossings), median of {reps}: {dt1:.2f} s"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU (--gpus 1); the library has no "
                                   "multi-GPU path"}))
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
        summary, details = sweeps(tomo, ts, only=tuple(args.sweep_only), tune=not args.sweep_no_autotune)
        print(json.dumps({"sweep": details["points"]}), flush=True)
        return
    if args.euvi_only:
        _, _, _, e = euvi_step(tomo, ts, steps=args.steps)
        print(json.dumps({"euvi": e}), flush=True)
        return

    cb, h = headline(tomo, ts, args)
    out = {
        "metric": METRIC,
        "value": h["value"],
        "unit": "voxel-crossings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "COR1-like batched time-evolving inversion: 8 frames of 256^3 on [-4,4]^3 R_sun "
                               "(60 views of 512x512, annulus 1.4-4 R_sun kept, unit sphere masked, "
                               "lambda_t 10) + 64^3, 96^3, 128^3, 192^3 extras (16 views of 256x256 each), "
                               f"{args.iters} graph-captured batched CG iterations, lambda 1e-2",
                   "crossings_per_application": cb.cross, "applications_per_step": h["applications"],
                   "rays": h["rays"], "arithmetic": "f32 storage and vectors, f64 ray walk and dot products, "
                                                    "64-bit fixed-point P^T bins",
                   "autotuned": not args.no_autotune},
        "kernels": {"p_launches_ms": h["ms_p"], "k_batch_backproject_ms": h["ms_b"],
                    "project_crossings_per_s": h["cross_p"] / (h["ms_p"] * 1e-3),
                    "backproject_crossings_per_s": h["cross_b"] / (h["ms_b"] * 1e-3)},
        "roofline": roofline(h),
    }
    details = {"headline": {"tunings": cb.tunings, "final_rel_res": h["final_rel_res"],
                            "p_items": cb.batch.items(0), "pt_items": cb.batch.items(1),
                            "p_workgroups": cb.batch.items(2), "pt_workgroups": cb.batch.items(3)}}
    if args.headline_only:
        print(json.dumps(out), flush=True)
        return
    if not args.no_sequential:
        ms_seq = sequential(tomo, cb, args.iters)
        out["batched"] = {"ms_batched": h["ms_step"], "ms_sequential": ms_seq, "speedup": ms_seq / h["ms_step"]}
        log("sequential solves done")
    del cb
    torch.cuda.empty_cache()
    if not args.no_probes:
        out["achievable"] = probes()
    wl = dg = y = None
    if not args.no_euvi:
        wl, dg, y, out["euvi"] = euvi_step(tomo, ts)
        log("EUVI-like step done")
    if not args.no_learned:
        out["time_to_rel_res_1e-3"], details["learned"] = learned_vs_plain(tomo, ts)
        log("learned vs plain done")
    if not args.no_obstacle and wl is not None:
        out["obstacle"] = obstacle_euvi(tomo, ts, wl, y)
        log("obstacle variant done")
    if not args.no_thomson:
        out["thomson"] = thomson_cor1(tomo, ts)
        log("Thomson operators done")
    if not args.no_height_gain and wl is not None:
        out["height_gain"] = height_gain_euvi(tomo, ts, wl, y)
        log("two instruments with the height-weighted prior done")
    if not args.no_configs:
        out["configs"], details["configs"] = per_config(tomo, ts)
        log("per-configuration P and P^T done")
    if not args.no_sweep:
        out["sweep"], details["sweep"] = sweeps(tomo, ts, tune=not args.sweep_no_autotune)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ts, args.cpu_reps)
        log("cpu baseline done")
    try:
        os.makedirs(os.path.dirname(args.details), exist_ok=True)
        with open(args.details, "w") as fh:
            json.dump(details, fh, indent=1, default=float)
        out["details"] = os.path.relpath(args.details, ROOT)
    except OSError as e:
        log(f"details not written: {e}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
