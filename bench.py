"""SupPCG benchmark on one MI355X.

Workload: 512x512 image, 720 angles over [0, pi), 725 unit bins; random-ellipse
phantom (20 ellipses, seed 1) with 0.5% Gaussian noise; K = 1, a = 0.5,
gamma = 0.5 (first trial step 0.5^k), ramp-Hamming preconditioner
(mu = 1e-5, rho = 0.8).  One step = one SupPCG iteration (S_TV + U_PCG: the
projections R x_{k+1/2} and R z, one backprojection R^T, one preconditioner
apply, TV work and the CG updates; U_PCG's h = A p enters through R p, which
the solver carries).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 100] [--warmup 5] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = dict(name="ct512", rows=512, cols=512, n_angles=720, n_bins=725, ellipses=20, seed=1,
                noise=0.005)
# Nonzero entries of R (strictly positive chord lengths), counted with the
# oracle's closed form by tests/golden/count_nnz.py.
NNZ_CT512 = 240_840_802
NNZ_2048 = 10_945_428_176
# Non-packed VALU issue rate: 256 CUs x 64 lanes x 2.4 GHz lane-operations/s.
# The published 157.3 TFLOP/s FP32 counts an FMA as 2 flops on 2-wide packed
# lanes; these kernels are float64 (FP64 FMA issues at the same non-packed
# rate, 78.6 TFLOP/s = 39.3 T FMA/s) and generate no packed FP32.
PEAK_VALU_OPS = 256 * 64 * 2.4e9
# HBM3E peak of one MI355X, bytes/s
PEAK_HBM = 8e12
# Algorithmic work of R and R^T: the fewest lane-operations a matrix-free
# projector can spend on one nonzero weight -- form the ray-pixel offset,
# evaluate the chord length from it, address the gathered value, and
# multiply-add it into the sum: 4 per nonzero, i.e. 4 nnz per call (24.5 us of
# VALU issue at this workload).  A kernel that does the work cannot issue
# fewer, so roofline.frac cannot exceed 1.
OPS_PER_NNZ = 4
# Hardware counters of the kernels at this workload, as measured by the
# rocprofv3 runs summarised in profiles/counters_ct512.md (taken at the commit
# named below; re-measure after changing a kernel).  VALU wave-instructions per
# launch (SQ_INSTS_VALU, 64 lane-operations each) and bytes between L2 and the
# memory fabric per launch (FETCH_SIZE + WRITE_SIZE, scaled by the counters of
# a 64 MiB device copy).  R^T: its float64 (residual) sinogram form, the one
# the loop body runs.
COUNTERS = {"measured_at": "kernels of fa5dc61",
            "valu_instr": {"project": 2.696e7, "backproject": 3.275e7},
            "traffic_bytes": {"project": 43.22e6, "backproject": 14.46e6}}
# The vector L1's access rate, the limit the gathers of both kernels run into
# (profiles/memory_pipe_ct512.md, same kernels):
# TCP_TOTAL_CACHE_ACCESSES per launch and per compute unit and cycle of the
# kernel's own run (about one access per CU and cycle is the L1's rate; R^T:
# its float64 form, as above).
L1_ACCESS = {"measured_at": "kernels of fa5dc61",
             "per_launch": {"project": 5.702e7, "backproject": 5.58e7},
             "per_cu_per_cycle": {"project": 1.01, "backproject": 0.84}}


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--reps", type=int, default=20, help="timed calls per operator")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--eager", action="store_true", help="launch the loop eagerly, no graph")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-slice batched run")
    ap.add_argument("--learned-steps", type=int, default=2000,
                    help="Adam steps of the 64^2 learned preconditioner (shorter for profiling)")
    ap.add_argument("--learned-seeds", type=int, default=32, help="evaluation seeds from 100")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip training the learned preconditioner and its time-to-target")
    ap.add_argument("--batch-iters", type=int, default=50)
    ap.add_argument("--no-quality", action="store_true", help="skip the selective-error curves")
    ap.add_argument("--no-stored", action="store_true", help="skip the stored-matrix products")
    ap.add_argument("--stored-sides", type=int, nargs="+", default=[64, 128, 256, 512, 1024])
    ap.add_argument("--quality-iters", type=int, default=100)
    ap.add_argument("--large", action="store_true",
                    help="also run 8 slices of 2048^2 x 2048 x 2899 (about a minute of phantom setup)")
    ap.add_argument("--large-iters", type=int, default=200)
    ap.add_argument("--large-quick-iters", type=int, default=20,
                    help="iterations of the short 2048^2 batch run made without --large")
    ap.add_argument("--no-large", action="store_true", help="skip the short 2048^2 batch run")
    ap.add_argument("--learned512", action="store_true",
                    help="also train and judge the learned preconditioner at 512^2 x 720 x 725")
    return ap.parse_args()


def batched_run(sp, torch, iters):
    """64 mixed slices (sides 256..1024, 1.4 x side angles, ceil(side sqrt 2) + 1
    bins) in one batched solve, against the same slices solved one by one."""
    from synth import batched_slices, random_ellipses
    work = batched_slices(64, seed=2)
    geoms = [sp.Geometry(w.rows, w.cols, w.n_angles, w.n_bins) for w in work]
    bs = []
    for w, g in zip(work, geoms):
        img, rng = random_ellipses(w.rows, w.cols, w.n_ellipses, w.seed)
        x = torch.from_numpy(img.astype(np.float32)).cuda()
        b = sp.sp_project(g, x)
        noise = torch.from_numpy(rng.standard_normal(g.m).astype(np.float32)).cuda()
        bs.append((b + w.noise_frac * float(b.max()) * noise.reshape(b.shape)).contiguous())
    kw = dict(K=1, a=0.5, gamma=0.5, mu=1e-5, rho=0.8)
    sp.sp_suppcg_solve_batched(geoms, bs, graph=True, autotune=True, max_iter=2, **kw)  # layout + tuning
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    res = sp.sp_suppcg_solve_batched(geoms, bs, graph=True, max_iter=iters, **kw)
    e1.record()
    torch.cuda.synchronize()
    t_batch = e0.elapsed_time(e1) / 1e3
    e0.record()
    for g, b in zip(geoms, bs):
        sp.sp_suppcg_solve(g, b, None, graph=True, max_iter=iters, trace=False, **kw)
    e1.record()
    torch.cuda.synchronize()
    t_seq = e0.elapsed_time(e1) / 1e3
    shapes = {f"{g.rows}x{g.cols}x{g.n_angles}x{g.n_bins}": {"parts": p_, "px": x_}
              for g, p_, x_ in sp.tuning_list() if g in set(geoms)}
    return {"workload": "64 slices, sides {256,384,512,768,1024} (seed 2), 1.4 x side angles, "
                        "ceil(side sqrt 2)+1 bins, SupPCG K=1, ramp-Hamming M",
            "tuned_shapes": shapes,
            "iterations": iters, "slice_iterations_per_s": round(64 * iters / t_batch, 2),
            "one_by_one_slice_iterations_per_s": round(64 * iters / t_seq, 2),
            "speedup_vs_one_by_one": round(t_seq / t_batch, 3),
            "all_k": sorted(set(r.k for r in res)), "tuning": sp.batch_tuning()}


# Table 1's parameters per method, and the defaults of the main workload
QUALITY_PRESETS = {
    "table1": {"SupPCG": dict(K=40, a=1 - 1e-5, gamma=1e-2, mu=1e-5, rho=0.8),
               "PCG": dict(K=0, mu=1e-3, rho=0.6),
               "SupCG": dict(K=40, a=1 - 1e-5, gamma=5e-2, precond="none"),
               "CG": dict(K=0, precond="none")},
    "default": {"SupPCG": dict(K=1, a=0.5, gamma=0.5, mu=1e-5, rho=0.8),
                "PCG": dict(K=0, mu=1e-5, rho=0.8),
                "SupCG": dict(K=1, a=0.5, gamma=0.5, precond="none"),
                "CG": dict(K=0, precond="none")},
}
QUALITY_WORKLOADS = {"ct512": (512, 512, 720, 725, 20, 1, 0.005),
                     "paper243": (243, 243, 360, 345, 20, 3, 0.01)}


def quality_run(sp, torch, iters):
    """Iteration-wise and time-wise selective-error curves (eq. (4.1), the
    ellipse of Section 4.2 scaled to the image width) of SupPCG, PCG, SupCG and
    CG, each under Table 1's parameters and under the defaults, and of ART,
    SupART and BlobART under Table 1's (40 cycles), at 512^2 x 720 x 725 and at the
    paper's shape (243^2 x 360 x 345); graph-replayed loop bodies, HIP events
    between them."""
    from synth import noisy_data, random_ellipses, unit_noise
    marks = sorted(set([0, 1, 2, 3, 4, 5] + list(range(10, iters + 2, 5)) + [iters + 1]))
    out = {}
    for wname, (rows, cols, A, B, ne, seed, frac) in QUALITY_WORKLOADS.items():
        g = sp.Geometry(rows, cols, A, B)
        img, rng = random_ellipses(rows, cols, ne, seed)
        x_true = torch.from_numpy(img.astype(np.float32)).cuda()
        b_exact = sp.sp_project(g, x_true)
        b_np = noisy_data(b_exact.cpu().numpy().ravel(), unit_noise(rng, g.m), frac)
        b = torch.from_numpy(b_np.astype(np.float32).reshape(A, B)).cuda()
        res_w = {"geometry": f"{rows}x{cols}, {A} angles, {B} bins; {ne} ellipses (seed {seed}), "
                             f"{frac * 100:g}% noise",
                 "ellipse_semi_axes": [round(v, 3) for v in sp.paper_se_axes(g)]}
        for pname, preset in QUALITY_PRESETS.items():
            for method, kw in preset.items():
                sp.sp_suppcg_solve(g, b, None, max_iter=2, graph=True, trace=False, **kw)
                r = sp.sp_suppcg_solve(g, b, None, max_iter=iters, graph=True, se_ref=x_true,
                                       timing=True, **kw)
                se, t = r.trace["se"], r.trace["t_ms"]
                kb = int(np.nanargmin(se))
                res_w[f"{method}/{pname}"] = {
                    "params": {k: v for k, v in kw.items()},
                    "best": {"iteration": kb, "se": round(float(se[kb]), 6),
                             "ms": round(float(t[kb]), 3)},
                    "ms_total": round(float(t[-1]), 3),
                    "curve": [[k, round(float(se[k]), 6), round(float(t[k]), 3)]
                              for k in marks if k < len(se)]}
        # ART, SupART and BlobART (Section 3.4) under Table 1's parameters
        art_iters = min(iters, 40)
        amarks = [k for k in marks if k <= art_iters]
        for method, kw in (("ART", dict(K=0, r=5.0, lam=1e-2)),
                           ("SupART", dict(K=10, a=1 - 1e-5, gamma=1e-2, r=5.0, lam=5e-2)),
                           ("BlobART", dict(r=5.0, lam=1e-2))):
            solve = sp.sp_blobart_solve if method == "BlobART" else sp.sp_supart_solve
            solve(g, b, max_iter=1, **kw)
            r_ = solve(g, b, max_iter=art_iters, se_ref=x_true, timing=True, **kw)
            se, t = r_.trace["se"], r_.trace["t_ms"]
            kb = int(np.nanargmin(se))
            res_w[f"{method}/table1"] = {
                "params": kw, "best": {"iteration": kb, "se": round(float(se[kb]), 6), "ms": round(float(t[kb]), 3)},
                "ms_total": round(float(t[-1]), 3), "ms_per_cycle": round(float(t[-1]) / art_iters, 3),
                "curve": [[k, round(float(se[k]), 6), round(float(t[k]), 3)] for k in amarks if k < len(se)]}
        out[wname] = res_w
    return {"iterations": iters, "curve_columns": ["iteration k", "SE(x_k)", "ms to x_k"],
            "workloads": out}


def stored_run(sp, torch, reps, sides):
    """Stored-weight R and R^T (CSR in HBM, 8 bytes per nonzero per side)
    against the matrix-free kernels, at square images of the given sides with
    round(720 / 512 * side) angles and round(725 / 512 * side) bins (the 512^2
    workload's shape scaled).  Times are HIP-event means over `reps` calls."""
    from synth import random_ellipses
    L = sp.api.L
    ctx = sp.context(0)
    rows_out = []
    for side in sides:
        A = int(round(720 / 512 * side))
        B = int(round(725 / 512 * side))
        g = sp.Geometry(side, side, A, B)
        img, _ = random_ellipses(side, side, 20, 1)
        x = torch.from_numpy(img.astype(np.float32)).cuda()
        y = sp.sp_project(g, x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M = sp.StoredMatrix(g)
        t_build = time.perf_counter() - t0
        nnz, nbytes = M.info()
        yo = torch.empty_like(y)
        xo = torch.empty_like(x)

        def timed(fn, kind):
            fn()
            ctx.profile_enable(True)
            for _ in range(reps):
                fn()
            ms, cnt = ctx.profile_read(kind)
            ctx.profile_enable(False)
            return ms / max(cnt, 1)

        ms_sR = timed(lambda: M.project(x, yo), L.SP_PROF_STORED_PROJECT)
        ms_sRT = timed(lambda: M.backproject(y, xo), L.SP_PROF_STORED_BACKPROJECT)
        ms_R = timed(lambda: sp.sp_project(g, x, yo), L.SP_PROF_PROJECT)
        ms_RT = timed(lambda: sp.sp_backproject(g, y, xo), L.SP_PROF_BACKPROJECT)
        n, m = side * side, A * B
        # algorithmic bytes of one stored product: 8 per nonzero of the matrix
        # side it streams, its row lengths and slice offsets, the input vector
        # once and the output (padding entries are never read)
        bytes_R = 8 * nnz + 4 * m + 8 * (m // 64 + 1) + 4 * n + 4 * m
        bytes_RT = 8 * nnz + 4 * n + 8 * (n // 64 + 1) + 4 * m + 4 * n
        rows_out.append({
            "geometry": f"{side}x{side}, {A} angles, {B} bins", "nnz": nnz,
            "matrix_GB_both_sides": round(nbytes / 1e9, 3), "build_s": round(t_build, 3),
            "stored_ms": {"R": round(ms_sR, 4), "RT": round(ms_sRT, 4)},
            "matrix_free_ms": {"R": round(ms_R, 4), "RT": round(ms_RT, 4)},
            "stored_GBps": {"R": round(bytes_R / (ms_sR / 1e3) / 1e9, 1),
                            "RT": round(bytes_RT / (ms_sRT / 1e3) / 1e9, 1)},
            "stored_frac_of_8TBps": {"R": round(bytes_R / (ms_sR / 1e3) / PEAK_HBM, 4),
                                     "RT": round(bytes_RT / (ms_sRT / 1e3) / PEAK_HBM, 4)},
            "stored_over_matrix_free": {"R": round(ms_sR / ms_R, 3), "RT": round(ms_sRT / ms_RT, 3)}})
        M.close()
        del M
        torch.cuda.synchronize()
    return {"reps": reps, "sizes": rows_out}


def large_run(sp, torch, iters, learned=True):
    """8 slices of 2048^2 x 2048 angles x 2899 bins in one batched solve, plus
    standalone R and R^T timings at that geometry; with `learned`, the learned
    preconditioner retrained at that geometry and its time to target."""
    from synth import large_batch, noisy_data, random_ellipses, unit_noise
    work = large_batch(8)
    geoms = [sp.Geometry(w.rows, w.cols, w.n_angles, w.n_bins) for w in work]
    bs = []
    for w, g in zip(work, geoms):
        img, rng = random_ellipses(w.rows, w.cols, w.n_ellipses, w.seed)
        x = torch.from_numpy(img.astype(np.float32)).cuda()
        b_exact = sp.sp_project(g, x).cpu().numpy().ravel()
        b = noisy_data(b_exact, unit_noise(rng, g.m), w.noise_frac).astype(np.float32)
        bs.append(torch.from_numpy(b.reshape(g.n_angles, g.n_bins)).cuda())
        log(f"large slice {w.name} ready")
    ctx = sp.context(0)
    L = sp.api.L
    x = torch.from_numpy(random_ellipses(2048, 2048, 50, 5000)[0].astype(np.float32)).cuda()
    y = torch.empty((2048, 2899), device="cuda")
    xo = torch.empty((2048, 2048), device="cuda")
    def op_ms(fn, kind):
        fn()
        ctx.profile_enable(True)
        for _ in range(3):
            fn()
        ms, n = ctx.profile_read(kind)
        ctx.profile_enable(False)
        return ms / max(n, 1)
    ms_r = op_ms(lambda: sp.sp_project(geoms[0], x, y), L.SP_PROF_PROJECT)
    ms_rt = op_ms(lambda: sp.sp_backproject(geoms[0], bs[0], xo), L.SP_PROF_BACKPROJECT)
    kw = dict(K=1, a=0.5, gamma=0.5, mu=1e-5, rho=0.8)
    sp.sp_suppcg_solve_batched(geoms, bs, graph=True, autotune=True, max_iter=2, **kw)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    res = sp.sp_suppcg_solve_batched(geoms, bs, graph=True, max_iter=iters, **kw)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3
    n, m = 2048 * 2048, 2048 * 2899
    eq = 8 * NNZ_2048 + 4 * n + 4 * m
    out = {"workload": "8 slices 2048x2048, 2048 angles, 2899 bins, 50 ellipses (seeds 5000-5007), "
                       "noise 0.25-2%, SupPCG K=1, ramp-Hamming M",
           "iterations": iters, "batch_iterations_per_s": round(iters / t, 3),
           "slice_iterations_per_s": round(8 * iters / t, 3),
           "R_ms": round(ms_r, 3), "RT_ms": round(ms_rt, 3), "nnz_per_slice": NNZ_2048,
           "stored_matrix_equivalent": {"R_GBps": round(eq / (ms_r / 1e3) / 1e9, 1),
                                        "RT_GBps": round(eq / (ms_rt / 1e3) / 1e9, 1)},
           "all_k": sorted(set(r.k for r in res))}
    if not learned:
        return out
    # learned preconditioner retrained at this geometry on crop interiors, then
    # time to the plain run's f and TV at loop body 200 on the first slice
    from paper_1807_10151_amd import learned_train as lt
    cfg = lt.TrainConfig(n_ellipses=50, noise=0.005)
    tr = lt.train_crops(geoms[0], cfg, lt.CropConfig(), log_every=500)
    log("learned preconditioner trained at 2048^2")
    ttt = lt.time_to_target(geoms[0], tr.net, [5000], cfg, plain_iters=200, max_iters=400, reps=1)[0]
    learned = {"train_s": round(tr.seconds, 2), "probe_s": round(tr.probe_seconds, 2),
               "loss_first_last": [round(tr.losses[0][1], 4), round(tr.losses[-1][1], 4)],
               "plain_iterations": 200, "plain_s": round(ttt["plain_s"], 3),
               "learned_iterations_to_f": ttt["k_f"], "learned_iterations_to_tv": ttt["k_tv"],
               "learned_iterations_to_both": ttt["k_both"],
               "learned_s_to_both": (round(ttt["learned_s"], 3) if ttt["learned_s"] else None),
               "learned_f_at_200_over_target": round(ttt["learned_f_at_plain_iters"] / ttt["f_star"], 4)}
    out["time_to_target_seed_5000"] = learned
    return out


def learned512_run(sp):
    """The learned preconditioner at the 512^2 x 720 x 725 geometry: trained on
    4,096 crop interiors (96^2, margin 8) of 64 Gaussian images and 64 gradient
    snapshots g_{k+1/2} (k = 1..8, phantom seeds 10-17), then time to the plain
    run's f and TV at loop body 100 on seeds 100-107."""
    from paper_1807_10151_amd import learned_train as lt
    g = sp.Geometry(512, 512, 720, 725)
    cfg = lt.TrainConfig(n_ellipses=20, noise=0.005)
    cc = lt.CropConfig(crops_per_image=32, n_gauss_images=64, krylov_seeds=tuple(range(10, 18)),
                       krylov_per_seed=8, n_ellipses=20, noise=0.005)
    tr = lt.train_crops(g, cfg, cc, log_every=500)
    log("learned preconditioner trained at 512^2")
    rows = lt.time_to_target(g, tr.net, list(range(100, 108)), cfg, reps=1)
    reached = [r for r in rows if r["k_both"] is not None]
    return {"workload": "512x512, 720 angles, 725 bins, 20 ellipses, 0.5% noise; eval seeds 100-107",
            "train_s": round(tr.seconds, 2), "probe_s": round(tr.probe_seconds, 2),
            "loss_first_last": [round(tr.losses[0][1], 4), round(tr.losses[-1][1], 4)],
            "plain_iterations": 100,
            "learned_iterations_to_f": [r["k_f"] for r in rows],
            "learned_iterations_to_tv": [r["k_tv"] for r in rows],
            "learned_reached_f_and_tv_within_400": f"{len(reached)}/{len(rows)}",
            "learned_f_at_100_over_target": [round(r["learned_f_at_plain_iters"] / r["f_star"], 4)
                                             for r in rows],
            "plain_ms_median": round(1e3 * float(np.median([r["plain_s"] for r in rows])), 3),
            "learned_ms_to_both_median": (round(1e3 * float(np.median([r["learned_s"] for r in reached])), 3)
                                          if reached else None),
            "fallbacks": int(sum(r["fallbacks"] for r in rows))}


def learned_run(sp, steps=2000, n_seeds=32):
    """Train M = C^T diag(softplus(d)) C on the 64x64 / 90-angle geometry and
    compare its time to the plain (Fourier M) run's f and TV at loop body 100."""
    from paper_1807_10151_amd import learned_train as lt
    g = sp.Geometry(64, 64, 90, 91)
    cfg = lt.TrainConfig(steps=steps)
    res = lt.train(g, cfg, log_every=500)
    rows = lt.time_to_target(g, res.net, list(range(100, 100 + n_seeds)), cfg, reps=1)
    kf = [r["k_f"] for r in rows]
    kb = [r["k_both"] for r in rows]
    reached = [r for r in rows if r["k_both"] is not None]
    return {"workload": f"64x64, 90 angles, 91 bins, 5 ellipses, 1% noise; eval seeds 100-{99 + n_seeds}",
            "adam_steps": steps,
            "train_s": round(res.seconds, 3), "probe_s": round(res.probe_seconds, 3),
            "loss_first_last": [round(res.losses[0][1], 5), round(res.losses[-1][1], 5)],
            "plain_iterations": 100,
            "learned_iterations_to_f_median": float(np.median([k if k else 10 ** 6 for k in kf])),
            "learned_reached_f_and_tv_within_400": f"{len(reached)}/{len(rows)}",
            "learned_iterations_to_both_median": (float(np.median([r["k_both"] for r in reached]))
                                                  if reached else None),
            "plain_ms_median": round(1e3 * float(np.median([r["plain_s"] for r in rows])), 3),
            "learned_ms_to_both_median": (round(1e3 * float(np.median([r["learned_s"] for r in reached])), 3)
                                          if reached else None),
            "fallbacks": int(sum(r["fallbacks"] for r in rows))}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_r_worker(lo, hi, x, y, reps, barrier, out):
    """One host worker of the all-cores oracle leg: the rows of R for angles
    [lo, hi) (closed-form CSR, built before timing) and their transpose."""
    import scipy.sparse as sps

    from oracle import closed_form
    from oracle.geometry import Geometry as OG
    og = OG(WORKLOAD["rows"], WORKLOAD["cols"], WORKLOAD["n_angles"], WORKLOAD["n_bins"])
    Rw = sps.vstack([closed_form.angle_block(og, a) for a in range(lo, hi)], format="csr")
    RTw = Rw.T.tocsr()
    yw = y[lo * og.n_bins:hi * og.n_bins]
    barrier.wait()
    for _ in range(reps):
        Rw @ x
    barrier.wait()
    part = None
    for _ in range(reps):
        part = RTw @ yw
    barrier.wait()
    out.put((lo, part))


def _cpu_all_cores(x, y, reps=3):
    """R and R^T of the oracle at full size on all host cores: worker processes
    hold blocks of R by angle (CSR row blocks) and of R^T by the same angles
    (column blocks, partial images summed by the parent).  Returns (seconds per
    R, seconds per R^T, workers)."""
    import multiprocessing as mp
    nw = max(1, min(os.cpu_count() or 1, 16))
    A = WORKLOAD["n_angles"]
    bounds = [(A * i // nw, A * (i + 1) // nw) for i in range(nw)]
    ctx = mp.get_context("spawn")
    barrier = ctx.Barrier(nw + 1)
    out = ctx.Queue()
    procs = [ctx.Process(target=_cpu_r_worker, args=(lo, hi, x, y, reps, barrier, out))
             for lo, hi in bounds]
    for p in procs:
        p.start()
    barrier.wait(timeout=600)                 # every block built
    t0 = time.perf_counter()
    barrier.wait(timeout=600)
    t1 = time.perf_counter()
    barrier.wait(timeout=600)
    parts = [out.get(timeout=600) for _ in procs]
    img = np.zeros_like(x)
    for _, part in sorted(parts, key=lambda t: t[0]):
        img += part
    t2 = time.perf_counter()
    for p in procs:
        p.join(timeout=60)
    return (t1 - t0) / reps, (t2 - t1) / reps, nw


def cpu_baseline(img, b):
    """The float64 oracle on the host.  All cores: R and R^T at full size split
    over worker processes by angle; M, S_TV and the vector work as the oracle
    runs them (NumPy, one thread).  One core: R and R^T on a sample of angles
    scaled to all angles.  One iteration = 2 R + 2 R^T + M + S_TV + vector work."""
    import scipy.sparse as sps

    from oracle import closed_form, precond, suppcg
    from oracle.geometry import Geometry as OG

    og = OG(WORKLOAD["rows"], WORKLOAD["cols"], WORKLOAD["n_angles"], WORKLOAD["n_bins"])
    x = img.astype(np.float64).ravel()
    y = b.astype(np.float64).ravel()
    xi = img.astype(np.float64)
    t0 = time.perf_counter()
    precond.apply(xi, 1e-5, 0.8)
    t_m = time.perf_counter() - t0
    t0 = time.perf_counter()
    suppcg.s_tv(xi, 0, suppcg.TVParams(1, 0.5, 0.5))
    t_stv = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(5):
        v = x * 0.5 + x
        float(v @ x)
    t_vec = (time.perf_counter() - t0) / 5 * 2
    # one core, sampled angles
    n_sample = 36
    angles = np.linspace(0, og.n_angles - 1, n_sample).astype(int)
    Rs = sps.vstack([closed_form.angle_block(og, int(a)) for a in angles], format="csr")
    RsT = Rs.T.tocsr()
    ys = y.reshape(og.n_angles, og.n_bins)[angles].ravel()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        Rs @ x
    t_r1 = (time.perf_counter() - t0) / reps * (og.n_angles / n_sample)
    t0 = time.perf_counter()
    for _ in range(reps):
        RsT @ ys
    t_rt1 = (time.perf_counter() - t0) / reps * (og.n_angles / n_sample)
    it_1 = 2 * t_r1 + 2 * t_rt1 + t_m + t_stv + t_vec
    # all cores, full size
    t_r, t_rt, nw = _cpu_all_cores(x, y)
    it_n = 2 * t_r + 2 * t_rt + t_m + t_stv + t_vec
    return {"value": round(1.0 / it_n, 4), "unit": "iterations/s", "cores": nw, "kind": "oracle",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "sample": (f"float64 NumPy/SciPy oracle at 512^2 x 720 x 725: R and R^T (closed-form "
                       f"CSR, 240.8M nonzeros) in full on {nw} worker processes by angle block; "
                       f"M, S_TV and vector work single-threaded as the oracle runs them; one "
                       f"iteration = 2 R + 2 R^T + M + S_TV + vector work; R {t_r*1e3:.0f} ms, "
                       f"R^T {t_rt*1e3:.0f} ms, M {t_m*1e3:.0f} ms, S_TV {t_stv*1e3:.0f} ms"),
            "single_core": {"value": round(1.0 / it_1, 4), "cores": 1,
                            "sample": (f"R and R^T on {n_sample} of {og.n_angles} angles scaled "
                                       f"to all angles: R {t_r1*1e3:.0f} ms, R^T {t_rt1*1e3:.0f} ms")}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding of "
              "this path is a design note, not a measured configuration.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1807_10151_amd as sp
    from synth import noisy_data, random_ellipses, unit_noise

    dev = torch.device("cuda:0")
    w = WORKLOAD
    g = sp.Geometry(w["rows"], w["cols"], w["n_angles"], w["n_bins"])
    img, rng = random_ellipses(w["rows"], w["cols"], w["ellipses"], w["seed"])
    x_true = torch.from_numpy(img.astype(np.float32)).to(dev)
    b_exact = sp.sp_project(g, x_true)
    noise = unit_noise(rng, g.m)
    b_np = noisy_data(b_exact.cpu().numpy().ravel(), noise, w["noise"]).astype(np.float32)
    b = torch.from_numpy(b_np.reshape(g.n_angles, g.n_bins)).to(dev)
    torch.cuda.synchronize()

    ctx = sp.context(0)
    L = sp.api.L

    # plain 64 MiB device copy: reference dispatch for scaling the FETCH_SIZE /
    # WRITE_SIZE hardware counters of a profiled run
    calib_src = torch.ones(16 * 1024 * 1024, device=dev)
    calib_dst = torch.empty_like(calib_src)
    calib_dst.copy_(calib_src)
    torch.cuda.synchronize()
    del calib_src, calib_dst

    # --- operator timings: HIP events around each kernel, recorded by the library
    # on its stream (torch's current stream)
    def op_ms(fn, kind, reps):
        fn()
        ctx.profile_enable(True)
        for _ in range(reps):
            fn()
        ms, n = ctx.profile_read(kind)
        ctx.profile_enable(False)
        return ms / max(n, 1)

    yout = torch.empty((g.n_angles, g.n_bins), device=dev)
    xout = torch.empty((g.rows, g.cols), device=dev)
    ms_R = op_ms(lambda: sp.sp_project(g, x_true, yout), L.SP_PROF_PROJECT, args.reps)
    ms_RT = op_ms(lambda: sp.sp_backproject(g, b, xout), L.SP_PROF_BACKPROJECT, args.reps)
    ms_M = op_ms(lambda: sp.sp_precond_apply(g, xout, 1e-5, 0.8), L.SP_PROF_PRECOND, args.reps)

    # --- SupPCG iterations (timed region): the loop body captured once in a HIP
    # graph and replayed, the solver's production mode (--eager: launched one
    # by one).  Capture, instantiation and the initial steps are inside the
    # timed call.
    kw = dict(K=1, a=0.5, gamma=0.5, mu=1e-5, rho=0.8, trace=True)
    if args.warmup > 0:
        sp.sp_suppcg_solve(g, b, None, max_iter=args.warmup, graph=not args.eager, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    res = sp.sp_suppcg_solve(g, b, None, max_iter=args.steps, graph=not args.eager, **kw)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    value = args.steps / (ms_total / 1e3)
    # the same solve launched eagerly with every R, R^T, M and S_TV launch
    # bracketed by HIP events in the library (a graph cannot time its nodes)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    e0.record()
    sp.sp_suppcg_solve(g, b, None, max_iter=args.steps, **kw)
    e1.record()
    torch.cuda.synchronize()
    eager_value = args.steps / (e0.elapsed_time(e1) / 1e3)
    solve_ms = {name: ctx.profile_read(kind) for name, kind in
                (("project", L.SP_PROF_PROJECT), ("backproject", L.SP_PROF_BACKPROJECT),
                 ("precond", L.SP_PROF_PRECOND), ("s_tv", L.SP_PROF_TV),
                 ("iteration", L.SP_PROF_ITERATION))}
    ctx.profile_enable(False)

    bytes_equiv = 8 * NNZ_CT512 + 4 * g.n + 4 * g.m
    avg = {k: v[0] / max(v[1], 1) for k, v in solve_ms.items()}
    kernels = {}
    for name in ("project", "backproject"):
        ms = avg[name]
        ach = OPS_PER_NNZ * NNZ_CT512 / (ms / 1e3)
        instr = COUNTERS["valu_instr"][name]
        kernels[name] = {"ms": round(ms, 4), "launches": solve_ms[name][1],
                         "achieved": round(ach / 1e12, 4), "frac": round(ach / PEAK_VALU_OPS, 4),
                         "valu_issue": {"instr_per_launch": instr,
                                        "frac": round(instr * 64 / (ms / 1e3) / PEAK_VALU_OPS, 4)},
                         "traffic": COUNTERS["traffic_bytes"][name],
                         "l1_accesses": {"per_launch": L1_ACCESS["per_launch"][name],
                                         "per_cu_per_cycle": L1_ACCESS["per_cu_per_cycle"][name]}}
    dom_name = max(kernels, key=lambda k: kernels[k]["ms"])
    dom = kernels[dom_name]
    out = {
        "metric": "SupPCG iterations/s + R/R^T GB/s at 512\u00b2x720; time-to-target, learned vs plain",
        "value": round(value, 3),
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 arithmetic in R, R^T, M and the CG scalars; f32 data and sinograms",
        "data": "synthetic random-ellipse phantom (20 ellipses, seed 1), 0.5% Gaussian noise",
        "config": {"workload": "ct512: 512x512 image, 720 angles over [0,pi), 725 bins, "
                               "SupPCG K=1 a=0.5 gamma=0.5, ramp-Hamming M mu=1e-5 rho=0.8",
                   "iterations": args.steps,
                   "timed_loop": "eager launches" if args.eager else "loop body replayed from a HIP graph",
                   "eager_event_timed_iterations_per_s": round(eager_value, 3)},
        "roofline": {"bound": "alu", "kernel": dom_name,
                     "achieved": dom["achieved"], "peak": round(PEAK_VALU_OPS / 1e12, 4),
                     "unit": "T lane-ops/s (VALU; 4 per nonzero weight of R)",
                     "frac": dom["frac"], "traffic": dom["traffic"],
                     "kernels": kernels, "nnz": NNZ_CT512,
                     "counters_measured_at": COUNTERS["measured_at"],
                     "l1_accesses_measured_at": L1_ACCESS["measured_at"]},
        "in_solve_ms": {k: round(v, 4) for k, v in avg.items()},
        "operators_ms": {"project": round(ms_R, 4), "backproject": round(ms_RT, 4),
                         "precond": round(ms_M, 4)},
        # the bytes a stored-matrix (CSR) SpMV of the same R would stream per
        # call, over the matrix-free kernels' time: an equivalence, not HBM
        # traffic (the matrix-free kernels move a few MB per call)
        "stored_matrix_equivalent": {
            "bytes_per_call": bytes_equiv,
            "project_GBps": round(bytes_equiv / (avg["project"] / 1e3) / 1e9, 1),
            "backproject_GBps": round(bytes_equiv / (avg["backproject"] / 1e3) / 1e9, 1)},
        "solve": {"k": res.k, "status": res.status_name, "wall_s": round(wall, 4),
                  "f_last": float(res.trace["f_half"][-1]) if len(res.trace["f_half"]) else None,
                  "ell_last": int(res.trace["ell"][-1]) if len(res.trace["ell"]) else None},
    }
    log("main solve done")
    # the launch-shape landscape at this workload (after the timed runs, which
    # use the default shapes; later parts of the run use the tuned ones)
    tuned = sp.tune_shapes(g)
    out["shape_tuning"] = {"parts": tuned["parts"], "px": tuned["px"],
                           "R_ms_by_parts": {str(k): round(v, 4) for k, v in tuned["R_ms"].items()},
                           "RT_ms_by_px": {str(k): round(v, 4) for k, v in tuned["RT_ms"].items()},
                           "note": "best of 5 standalone calls each, padding/prep launch included"}
    if not args.no_batch:
        out["batched"] = batched_run(sp, torch, args.batch_iters)
        log("batched run done")
    if args.learned512:
        out["learned_512"] = learned512_run(sp)
        log("learned preconditioner at 512^2 judged")
    if args.large:
        out["large"] = large_run(sp, torch, args.large_iters)
        log("2048^2 batch done")
    elif not args.no_large:
        # a short run of the 8 x 2048^2 batch (the full one, with the learned
        # preconditioner retrained there, is --large)
        out["large"] = large_run(sp, torch, args.large_quick_iters, learned=False)
        log("2048^2 batch (short) done")
    if not args.no_stored:
        out["stored_matrix"] = stored_run(sp, torch, args.reps, args.stored_sides)
        log("stored-matrix products timed")
    if not args.no_quality:
        out["quality_curves"] = quality_run(sp, torch, args.quality_iters)
        log("selective-error curves done")
    if not args.no_learned:
        out["time_to_target"] = learned_run(sp, args.learned_steps, args.learned_seeds)
        log("learned preconditioner trained and timed")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(img, b_np)
        log("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
