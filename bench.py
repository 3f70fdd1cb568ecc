"""Benchmark: relaxed-order mixed-precision GMRES on Stokes flow past 64 red
blood cells, against fixed-order FP64 GMRES.

Headline workload (synthetic, seeded): 64 Evans-Fung biconcave cells of 2048
flat triangles each (diameter 7.82 um), placed at random non-overlapping
positions and orientations in a 60 um cube (seed 0): 131072 panels, 524288
Gauss points, 393216 unknowns.  Stokes single layer, mu = 1, boundary data
u = (1, 0, 0) at every centroid; GMRES(50) to a relative residual of 1e-6.
A step is one relaxed solve: p from 16 down to p_min = 4 by the residual
(Eq. 17/19), FP32 P2P/expansions once eps_k >= 1e-5, FP64 Arnoldi, Givens and
true residuals, N_CRIT 112, M2L by rotation from p = 7 (the direct product
below); `value` = such solves per second with the inputs resident in device
memory.  Beside it: the fixed p = 16 FP64 solve (N_CRIT
192, the fastest for fixed p), p50 and max over the samples, the event-timed
roofline of the P2P and M2L kernels inside the timed solves, and the oracle's
CPU rate from a bounded row sample.

Secondary sections (outside the timed region): the Laplace sphere workloads
(2048 panels at fixed p = 10; 32768 panels with Y_l^m data, relaxed 12 -> 3 vs
fixed 12, per-order mat-vec times), the Stokes sphere of 8192 panels (drag
against 6 pi mu a U), the second-kind Laplace solve, and a serving stream of
512 requests through the request loop at three arrival rates calibrated from
the mean solo service time, with an 8 GB admission budget.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra] [--no-serving]
       python bench.py --timed-only            (the headline's timed region alone, for profiling)
       python bench.py --ncrit-sweep           (N_CRIT sweep of the Laplace 32768 and 64-cell cases)
       python bench.py --calibrate-copy        (a plain 1 GiB device copy, to scale HBM counters)
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

METRIC = "GMRES solve time & FMM matvec/s, relaxed vs fixed p at 1e-6 resid; p50/p99"
PEAK_FP32_VALU = 157.3e12  # MI355X published FP32 vector peak (packed)
PEAK_FP32_NONPACKED = 78.6e12
PEAK_FP64_VALU = 78.6e12
PEAK_HBM = 8.0e12  # bytes/s
TOL = 1e-6

# stage of the library's timing -> kernel that runs it (rocprofv3 names)
STAGE_KERNEL = {
    "stokes": {"p2p_fp32": "k_p2p<float, 1>", "p2p_fp64": "k_p2p<double, 1>",
               "m2l_fp32": "k_m2l_mfma<float, 4, 1|4>", "m2l_fp64": "k_m2l_stored<4>|k_m2l_valu<double, 4, 2>"},
    # M2L by rotation from p = 7 (the direct kernels below it)
    "stokes_rot": {"p2p_fp32": "k_p2p<float, 1>", "p2p_fp64": "k_p2p<double, 1>",
                   "m2l_fp32": "k_m2l_rot<float, 4, 2|4, 4> (p >= 7), k_m2l_mfma<float, 4, 1> (p < 7)",
                   "m2l_fp64": "k_m2l_rot<double, 4, 2, 4>"},
    "laplace": {"p2p_fp32": "k_p2p<float, 0>", "p2p_fp64": "k_p2p<double, 0>",
                "m2l_fp32": "k_m2l_mfma<float, 1, 1|4>", "m2l_fp64": "k_m2l_valu<double, 1, 8>"},
}


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def summary_ms(ts):
    """p50 and the tail of times ts (seconds) in ms: p99 from 100 samples on,
    below that the largest sample, labelled max."""
    a = 1e3 * np.asarray(ts, dtype=np.float64)
    out = {"n": int(a.size), "p50": float(np.percentile(a, 50)), "mean": float(a.mean())}
    if a.size >= 100:
        out["p99"] = float(np.percentile(a, 99))
    else:
        out["max"] = float(a.max())
    return out


M2L_MODES = {"fly": 0, "stored": 1, "rot": 2}  # params.m2l_stored

# source regions the HBM counter records were taken on: file, first marker, end marker
COUNTED_SOURCES = {
    "k_p2p<float, 1>": [("fmm.hip", "// P2P: one block per work unit", "// The downward pass of one leaf"),
                        ("tree.hip", "// P2P work units", "}  // namespace")],
    "k_p2p<float, 0>": [("fmm.hip", "// P2P: one block per work unit", "// The downward pass of one leaf"),
                        ("tree.hip", "// P2P work units", "}  // namespace")],
    "k_p2p<double, 1>": [("fmm.hip", "// P2P: one block per work unit", "// The downward pass of one leaf"),
                         ("tree.hip", "// P2P work units", "}  // namespace")],
    "k_near_spmv<float, false>": [("nearfield.hip", "// y_near = stored near field", "}  // namespace")],
    "k_near_spmv<double, false>": [("nearfield.hip", "// y_near = stored near field", "}  // namespace")],
    "k_m2l_mfma<float, 4, 1|4>": [("fmm.hip", "// M2L, in two passes.", "// LDS of k_m2l_mfma")],
    "k_m2l_stored<1>": [("fmm.hip", "// Pass 1 in FP64 from the stored operators",
                         "template <typename R> size_t m2l_mfma_shm")],
    "k_m2l_stored<4>": [("fmm.hip", "// Pass 1 in FP64 from the stored operators",
                         "template <typename R> size_t m2l_mfma_shm")],
    "k_m2l_rot<double, 4, 2, 4>": [("fmm.hip", "// M2L by rotation: the translation", "// LDS of k_m2l_rot"),
                                   ("rotations.cpp", "// Rotation operators", "}  // namespace fmmbem")],
    "k_m2l_rot<float, 4, 4, 4>": [("fmm.hip", "// M2L by rotation: the translation", "// LDS of k_m2l_rot"),
                                  ("rotations.cpp", "// Rotation operators", "}  // namespace fmmbem")],
    "k_m2l_rot<float, 4, 2, 4>": [("fmm.hip", "// M2L by rotation: the translation", "// LDS of k_m2l_rot"),
                                  ("rotations.cpp", "// Rotation operators", "}  // namespace fmmbem")],
    "k_m2l_rot<double, 1, 2, 4>": [("fmm.hip", "// M2L by rotation: the translation", "// LDS of k_m2l_rot"),
                                   ("rotations.cpp", "// Rotation operators", "}  // namespace fmmbem")],
}


def source_sha1(kernel: str) -> str:
    """Hash of the source of a kernel (and of what builds its work lists)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1506_05957_amd", "csrc")
    text = ""
    for fname, first, end in COUNTED_SOURCES[kernel]:
        with open(os.path.join(csrc, fname)) as f:
            s = f.read()
        a = s.index(first)
        text += s[a:s.index(end, a + len(first))]
    return hashlib.sha1(text.encode()).hexdigest()


def kernel_traffic(kernel: str, workload: str):
    """HBM bytes per launch of a kernel on a workload from the committed
    rocprofv3 counter records (FETCH_SIZE and WRITE_SIZE scaled by a plain
    copy), or None when there is no record whose kernel source is the
    current one (records taken before a change of the source are skipped)."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*hbm_counters*.md"))):
        try:
            with open(path) as f:
                text = f.read()
            recs = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        except (OSError, IndexError, ValueError):
            continue
        for rec in recs if isinstance(recs, list) else [recs]:
            if rec.get("kernel") != kernel or rec.get("workload", workload) != workload:
                continue
            try:
                if kernel not in COUNTED_SOURCES or rec.get("source_sha1") != source_sha1(kernel):
                    continue
            except (OSError, ValueError, KeyError):
                continue
            return float(rec["traffic_bytes_per_launch"])
    return None


def alu_roofline(stage, stage_name, kernel, workload, peak, bound="alu"):
    """Achieved algorithmic FLOP/s of one timed stage (HIP events on the
    stream its kernel runs on) against a vector-unit (or matrix-core) peak."""
    t_ms, launches, flops = stage
    if not launches:
        return None
    avg_s = t_ms / 1e3 / launches
    achieved = flops / launches / avg_s
    return {"bound": bound, "stage": stage_name, "kernel": kernel, "achieved": achieved / 1e12,
            "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak,
            "frac_of_nonpacked_fp32" if peak == PEAK_FP32_VALU else "frac_of_fp64":
                achieved / (PEAK_FP32_NONPACKED if peak == PEAK_FP32_VALU else PEAK_FP64_VALU),
            "traffic": kernel_traffic(kernel, workload), "avg_launch_us": avg_s * 1e6,
            "launches": launches, "flops_per_launch": flops / launches}


def timed_solves(fb, torch, ctx, b, x, sched, k, check=True):
    ts, reps = [], []
    for _ in range(k):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fb.fmmbem_solve_ctx(ctx, b, TOL, sched, x)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
        reps.append(r)
        if check:
            assert r["converged"] and r["rel_res_true"] <= TOL, r
    return ts, reps


def rep_summary(reps):
    return {"iterations": float(np.mean([r["iterations"] for r in reps])),
            "matvecs": float(np.mean([r["matvecs"] for r in reps])),
            "restarts": float(np.mean([r["restarts"] for r in reps])),
            "stalls": int(sum(r["stalls"] for r in reps)),
            "rel_res_true_max": float(max(r["rel_res_true"] for r in reps)),
            "converged": int(sum(int(r["converged"]) for r in reps))}


# ------------------------------------------------------------------ headline
def cells_headline(args, fb, syn, torch, dev):
    """The 64-cell Stokes case: relaxed mixed (N_CRIT 112) timed; fixed p = 16
    FP64 (N_CRIT 192) beside it."""
    m = syn.rbc_scene(64, 4, 0)
    nt = m.n_panels
    u = torch.tensor(np.tile([1.0, 0.0, 0.0], nt), device=dev)
    x = torch.empty_like(u)
    relaxed = fb.schedule(fb.STOKES, rule=fb.RELAX_BF, p_init=16, p_min=4, mixed=1, restart=50)
    fixed = fb.schedule(fb.STOKES, rule=fb.FIXED, p_init=16, p_min=16, mixed=0, restart=50)

    t0 = time.perf_counter()
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.STOKES, fb.params(ncrit=args.ncrit_relaxed, p_max=16,
                                                             m2l_stored=M2L_MODES[args.m2l]))
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    stats = fb.fmmbem_get_stats(ctx)
    print(f"bench: 64 cells built ({nt} panels, N_CRIT {args.ncrit_relaxed}) in {t_build:.2f}s: {stats}",
          file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        fb.fmmbem_solve_ctx(ctx, u, TOL, relaxed, x)
    torch.cuda.synchronize()

    # ---- timed region: K relaxed mixed-precision solves; the P2P and M2L
    # stages record HIP events on their own streams (two per mat-vec each)
    stages = ["p2p_fp32", "p2p_fp64", "m2l_fp32", "m2l_fp64"]
    fb.fmmbem_set_timing_stages(ctx, stages)
    fb.fmmbem_get_timing(ctx, reset=True)
    times, reps = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        r = fb.fmmbem_solve_ctx(ctx, u, TOL, relaxed, x)
        times.append(time.perf_counter() - ts)
        reps.append(r)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    stage = fb.fmmbem_get_timing(ctx, reset=True)
    fb.fmmbem_set_timing(ctx, False)
    for r in reps:
        assert r["converged"] and r["rel_res_true"] <= TOL, r
    x_relaxed = x.cpu().numpy()
    last = reps[-1]
    out = {"value": args.steps / t_total, "t_total": t_total, "times": times,
           "relaxed": {"solve_ms": summary_ms(times), **rep_summary(reps), "ncrit": args.ncrit_relaxed,
                       "p_history": [int(v) for v in last["p_hist"]],
                       "prec_history": [int(v) for v in last["prec_hist"]]},
           "stats": stats, "build_s": t_build, "mesh": m, "u": u, "x_relaxed": x_relaxed}

    # counter records hold per-launch bytes of one tree: the leaf size is part of the workload
    workload = f"stokes_64rbc_ncrit{args.ncrit_relaxed}"
    names = STAGE_KERNEL["stokes_rot" if args.m2l == "rot" else "stokes"]
    rl = {}
    for s in stages:
        # the rotation M2L runs on the matrix cores (dense peaks: FP32 157.3,
        # FP64 78.6 TFLOP/s, the same figures as the vector peaks used here)
        peak = PEAK_FP32_VALU if s.endswith("fp32") else PEAK_FP64_VALU
        bound = "mfma" if s.startswith("m2l") and args.m2l == "rot" else "alu"
        r = alu_roofline(stage[s], s, names[s], workload, peak, bound)
        if r:
            rl[s] = r
    dom = max(rl, key=lambda s: stage[s][0])
    out["roofline"] = rl[dom]
    out["roofline_by_stage"] = rl
    out["stage_ms_per_solve"] = {s: stage[s][0] / args.steps for s in stages}
    if args.timed_only:
        fb.fmmbem_destroy(ctx)
        return out

    # relaxed on the fixed schedule's tree (N_CRIT 192), for a same-tree factor
    ctx2 = fb.fmmbem_build(m.xyz, m.tri, fb.STOKES, fb.params(ncrit=args.ncrit_fixed, p_max=16,
                                                              m2l_stored=M2L_MODES[args.m2l]))
    fb.fmmbem_solve_ctx(ctx2, u, TOL, fixed, x)  # warm-up
    t_fix, r_fix = timed_solves(fb, torch, ctx2, u, x, fixed, args.fixed_reps)
    out["fixed"] = {"solve_ms": summary_ms(t_fix), **rep_summary(r_fix), "ncrit": args.ncrit_fixed}
    x_fixed = x.cpu().numpy()
    fb.fmmbem_solve_ctx(ctx2, u, TOL, relaxed, x)  # warm-up
    t_rs, r_rs = timed_solves(fb, torch, ctx2, u, x, relaxed, 3)
    out["relaxed_same_tree_as_fixed"] = {"solve_ms": summary_ms(t_rs), **rep_summary(r_rs),
                                         "ncrit": args.ncrit_fixed}
    fb.fmmbem_destroy(ctx2)
    # the two solutions agree in what the first-kind system fixes: the force on each cell
    F_rel = cell_forces(m, x_relaxed)
    F_fix = cell_forces(m, x_fixed)
    out["force_rel_diff_relaxed_vs_fixed"] = float(np.linalg.norm(F_rel - F_fix) / np.linalg.norm(F_fix))
    out["x_fixed"] = x_fixed

    # per-order mat-vec times (events, >= 100 reps after 5 warm-ups)
    out["matvec_ms"] = matvec_times(fb, torch, ctx, u, [(16, fb.FP64), (10, fb.FP32), (6, fb.FP32),
                                                        (4, fb.FP32)], args.matvec_reps)
    fb.fmmbem_destroy(ctx)
    return out


def cell_forces(m, t):
    """Force on each cell, sum of t_j S_j over its panels (cells are contiguous blocks of panels)."""
    v = m.xyz[m.tri]
    S = 0.5 * np.linalg.norm(np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), axis=1)
    f = t.reshape(-1, 3) * S[:, None]
    return f.reshape(64, -1, 3).sum(axis=1)


def matvec_times(fb, torch, ctx, x, orders, reps):
    """Event-timed mat-vecs on the current stream: {"p12_fp64": {p50, p99}, ...}."""
    y = torch.empty_like(x)
    out = {}
    for p, prec in orders:
        for _ in range(5):
            fb.fmmbem_matvec(ctx, p, prec, x, y)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            fb.fmmbem_matvec(ctx, p, prec, x, y)
            b.record()
        torch.cuda.synchronize()
        ts = [a.elapsed_time(b) / 1e3 for a, b in ev]
        s = summary_ms(ts)
        s["matvecs_per_s"] = 1e3 / s["mean"]
        out[f"p{p}_{'fp64' if prec == fb.FP64 else 'fp32'}"] = s
    return out


# ------------------------------------------------------------------ CPU leg
def cpu_baseline(args, fb, syn, head, sphere_mesh, sphere_x):
    """The oracle (dense FP64 CPU mat-vec with the same quadrature) on the
    host cores: 4096 sampled rows of the 64-cell operator applied to the GPU's
    relaxed solution, median of 3 runs, scaled to a full mat-vec and to the
    mat-vecs of a fixed-p solve; also the median of 3 full mat-vecs of the
    32768-panel Laplace operator.  The sampled rows also give the oracle's
    residual of the GPU solutions on those rows."""
    import oracle
    m = head["mesh"]
    nt = m.n_panels
    rng = np.random.default_rng(0)
    nrows = args.cpu_rows
    rows = np.sort(rng.choice(nt, nrows, replace=False))
    b_rows = np.tile([1.0, 0.0, 0.0], nrows)
    t_rows = []
    for _ in range(3):
        ts = time.perf_counter()
        y = oracle.matvec(oracle.STOKES, m.xyz, m.tri, head["x_relaxed"], rows=rows)
        t_rows.append(time.perf_counter() - ts)
    res_relaxed = float(np.linalg.norm(b_rows - y) / np.linalg.norm(b_rows))
    res_fixed = None
    if "x_fixed" in head:
        yf = oracle.matvec(oracle.STOKES, m.xyz, m.tri, head["x_fixed"], rows=rows)
        res_fixed = float(np.linalg.norm(b_rows - yf) / np.linalg.norm(b_rows))
    t_med = float(np.median(t_rows))
    t_mv = t_med * nt / nrows
    n_mv = head["fixed"]["matvecs"] if "fixed" in head else 70.0
    out = {"value": 1.0 / (t_mv * n_mv), "unit": "solves/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"dense FP64 oracle mat-vec of the 64-cell Stokes operator on {nrows} of {nt} sampled rows, "
                     f"median of 3 runs ({t_med:.2f}s), scaled to a full mat-vec ({t_mv:.1f}s) times the "
                     f"{n_mv:.0f} mat-vecs of the fixed-p solve",
           "matvec_s": t_mv, "rows_s_runs": t_rows,
           "oracle_rows_residual": {"relaxed_mixed": res_relaxed, "fixed_p16_fp64": res_fixed, "rows": nrows}}
    try:
        import multiprocessing
        out["cpu_model"] = open("/proc/cpuinfo").read().split("model name")[1].split(":")[1].split("\n")[0].strip()
        out["host_cpus"] = multiprocessing.cpu_count()
    except (OSError, IndexError):
        pass
    if sphere_mesh is not None and not args.no_cpu_sphere:
        t_full = []
        for _ in range(3):
            ts = time.perf_counter()
            oracle.matvec(oracle.LAPLACE, sphere_mesh.xyz, sphere_mesh.tri, sphere_x)
            t_full.append(time.perf_counter() - ts)
        out["laplace_sphere32768_full_matvec_s"] = {"median": float(np.median(t_full)), "runs": t_full}
    return out


# ------------------------------------------------------------------ secondary sections
def laplace_timed(args, fb, syn, torch, dev):
    """The relaxed mixed solves of the 32768-panel Laplace sphere alone (the
    configuration of laplace_sphere_32768, its five right-hand sides in turn,
    `--steps` rounds after `--warmup`), for profiling its kernels."""
    m = syn.sphere(6)
    rhs = [torch.tensor(syn.ylm_rhs(m, l, mm), device=dev) for l, mm in syn.ylm_orders(0)]
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE, fb.params(ncrit=64, p_max=12, near_stored=1, m2l_stored=2))
    x = torch.empty(m.n_panels, dtype=torch.float64, device=dev)
    s = fb.schedule(fb.LAPLACE, rule=fb.RELAX_BF, p_init=12, p_min=3, mixed=1)
    for _ in range(args.warmup):
        for b in rhs:
            fb.fmmbem_solve_ctx(ctx, b, TOL, s, x)
    ts = []
    for _ in range(args.steps):
        for b in rhs:
            t, r = timed_solves(fb, torch, ctx, b, x, s, 1)
            ts += t
    fb.fmmbem_destroy(ctx)
    return {"workload": "laplace_sl_sphere32768_ylm_tol1e-6", "relaxed_mixed_solve_ms": summary_ms(ts)}


def laplace_sphere_32768(args, fb, syn, torch, dev):
    """Laplace single layer, 32768-panel sphere, Y_l^m data (l = 0..4):
    relaxed mixed (12 -> 3), relaxed FP64 and fixed p = 12 FP64 solves with
    the stored near field and the rotation M2L (from p = 7); per-order mat-vec
    times; the rooflines of the FP64 M2L and of the near-field product."""
    m = syn.sphere(6)
    nt = m.n_panels
    orders = syn.ylm_orders(0)
    rhs = [torch.tensor(syn.ylm_rhs(m, l, mm), device=dev) for l, mm in orders]
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE, fb.params(ncrit=64, p_max=12, near_stored=1, m2l_stored=2))
    stats = fb.fmmbem_get_stats(ctx)
    x = torch.empty(nt, dtype=torch.float64, device=dev)
    scheds = {"relaxed_mixed": fb.schedule(fb.LAPLACE, rule=fb.RELAX_BF, p_init=12, p_min=3, mixed=1),
              "relaxed_fp64": fb.schedule(fb.LAPLACE, rule=fb.RELAX_BF, p_init=12, p_min=3, mixed=0),
              "fixed_p12_fp64": fb.schedule(fb.LAPLACE, rule=fb.FIXED, p_init=12, p_min=12, mixed=0)}
    for s in scheds.values():
        for b in rhs:
            fb.fmmbem_solve_ctx(ctx, b, TOL, s, x)
    out = {"workload": "laplace_sl_sphere32768_ylm_tol1e-6", "panels": nt, "ncrit": 64,
           "near_field": "stored", "m2l": "rot", "rhs": [f"Y_{l}^{mm}" for l, mm in orders]}
    fb.fmmbem_set_timing_stages(ctx, ["p2p_fp32", "m2l_fp64"])
    fb.fmmbem_get_timing(ctx, reset=True)
    for name, s in scheds.items():
        ts, reps = [], []
        for i in range(args.cmp_reps):
            t, r = timed_solves(fb, torch, ctx, rhs[i % len(rhs)], x, s, 1)
            ts += t
            reps += r
        out[name] = {"solve_ms": summary_ms(ts), **rep_summary(reps)}
        if name == "relaxed_mixed":
            stage = fb.fmmbem_get_timing(ctx, reset=True)
            out[name]["p_history_last"] = [int(v) for v in reps[-1]["p_hist"]]
    fb.fmmbem_set_timing(ctx, False)
    out["speedup_relaxed_vs_fixed"] = out["fixed_p12_fp64"]["solve_ms"]["p50"] / out["relaxed_mixed"]["solve_ms"]["p50"]
    # rooflines of the two dominant kernels, event-timed inside the relaxed
    # solves: the FP64 rotation M2L (p = 12) against the matrix-core peak with
    # the flops it applies, the near-field product against HBM
    rl = {}
    r = alu_roofline(stage["m2l_fp64"], "m2l_fp64", "k_m2l_rot<double, 1, 2, 4>", "laplace_sphere32768",
                     PEAK_FP64_VALU, "mfma")
    if r:
        rl["m2l_fp64"] = r
    t_ms, n, _ = stage["p2p_fp32"]
    if n:
        nbytes = stats["near_entries"] * 4 + 3 * 8 * nt
        avg = t_ms / 1e3 / n
        rl["near_fp32"] = {"bound": "hbm", "kernel": "k_near_spmv<float, false>", "achieved": nbytes / avg / 1e9,
                           "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": nbytes / avg / PEAK_HBM,
                           "traffic": kernel_traffic("k_near_spmv<float, false>", "laplace_sphere32768"),
                           "avg_launch_us": avg * 1e6, "launches": n, "bytes_per_launch": nbytes}
    out["roofline"] = rl
    out["matvec_ms"] = matvec_times(fb, torch, ctx, rhs[0], [(12, fb.FP64), (12, fb.FP32), (6, fb.FP32),
                                                             (3, fb.FP32)], args.matvec_reps)
    out["tree"] = {k: stats[k] for k in ("n_boxes", "n_leaves", "n_levels", "n_m2l", "n_p2p", "nnz_correction",
                                         "n_translations", "m2l_op_bytes", "near_entries", "device_bytes",
                                         "p2p_interactions")}
    fb.fmmbem_destroy(ctx)
    # P2P evaluated on the fly (event-timed kernel rate) on the same sphere
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE, fb.params(ncrit=64, p_max=12))
    y = torch.empty_like(x)
    for _ in range(3):
        fb.fmmbem_matvec(ctx, 3, fb.FP32, rhs[0], y)
    fb.fmmbem_set_timing_stages(ctx, ["p2p_fp32", "p2p_fp64"])
    fb.fmmbem_get_timing(ctx, reset=True)
    for _ in range(20):
        fb.fmmbem_matvec(ctx, 3, fb.FP32, rhs[0], y)
        fb.fmmbem_matvec(ctx, 3, fb.FP64, rhs[0], y)
    torch.cuda.synchronize()
    st = fb.fmmbem_get_timing(ctx, reset=True)
    fb.fmmbem_set_timing(ctx, False)
    pairs = stats["p2p_interactions"] - 4 * nt
    out["p2p_on_the_fly"] = {}
    for s, peak in (("p2p_fp32", PEAK_FP32_VALU), ("p2p_fp64", PEAK_FP64_VALU)):
        t_ms, n, fl = st[s]
        avg = t_ms / 1e3 / n
        out["p2p_on_the_fly"][s] = {"kernel_us": avg * 1e6, "interactions_per_s": pairs / avg,
                                    "tflops": fl / n / avg / 1e12, "frac": fl / n / avg / peak}
    fb.fmmbem_destroy(ctx)
    return out, m, rhs[0].cpu().numpy()


def laplace_sphere_2048(args, fb, syn, torch, dev):
    """Laplace single layer on the 2048-panel sphere, phi = 1 (exact density
    1): fixed p = 10 FP64, N_CRIT 64 (and the relaxed schedule beside it)."""
    m = syn.sphere(4)
    b = torch.ones(m.n_panels, dtype=torch.float64, device=dev)
    x = torch.empty_like(b)
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE, fb.params(ncrit=64, p_max=10))
    out = {"workload": "laplace_sl_sphere2048_phi1_tol1e-6", "panels": m.n_panels, "ncrit": 64}
    for name, s in (("fixed_p10_fp64", fb.schedule(fb.LAPLACE, rule=fb.FIXED, p_init=10, p_min=10, mixed=0)),
                    ("relaxed_mixed", fb.schedule(fb.LAPLACE, rule=fb.RELAX_BF, p_init=10, p_min=3, mixed=1))):
        fb.fmmbem_solve_ctx(ctx, b, TOL, s, x)
        ts, reps = timed_solves(fb, torch, ctx, b, x, s, args.cmp_reps)
        err = float(torch.linalg.norm(x - 1.0) / np.sqrt(m.n_panels))
        out[name] = {"solve_ms": summary_ms(ts), **rep_summary(reps), "density_rel_err_vs_exact": err}
    out["matvec_ms"] = matvec_times(fb, torch, ctx, b, [(10, fb.FP64)], args.matvec_reps)
    fb.fmmbem_destroy(ctx)
    return out


def stokes_sphere_8192(args, fb, syn, torch, dev):
    """Stokes single layer, unit sphere of 8192 panels translating at
    u = (1, 0, 0), mu = 1: relaxed mixed 16 -> 4 against fixed p = 16 FP64;
    drag against 6 pi mu a U."""
    m = syn.sphere(5)
    nt = m.n_panels
    u = torch.tensor(np.tile([1.0, 0.0, 0.0], nt), device=dev)
    x = torch.empty_like(u)
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.STOKES, fb.params(ncrit=64, p_max=16))
    v = m.xyz[m.tri]
    S = 0.5 * np.linalg.norm(np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]), axis=1)
    out = {"workload": "stokes_sl_sphere8192_translating_tol1e-6", "panels": nt, "unknowns": 3 * nt, "ncrit": 64}
    for name, s in (("relaxed_mixed", fb.schedule(fb.STOKES, rule=fb.RELAX_BF, p_init=16, p_min=4, mixed=1)),
                    ("fixed_p16_fp64", fb.schedule(fb.STOKES, rule=fb.FIXED, p_init=16, p_min=16, mixed=0))):
        fb.fmmbem_solve_ctx(ctx, u, TOL, s, x)
        ts, reps = timed_solves(fb, torch, ctx, u, x, s, args.cmp_reps)
        t = x.cpu().numpy().reshape(-1, 3)
        Fx = float((t[:, 0] * S).sum())
        out[name] = {"solve_ms": summary_ms(ts), **rep_summary(reps), "drag_Fx": Fx,
                     "drag_rel_err_vs_6pi": abs(abs(Fx) - 6 * np.pi) / (6 * np.pi)}
    out["speedup_relaxed_vs_fixed"] = out["fixed_p16_fp64"]["solve_ms"]["p50"] / out["relaxed_mixed"]["solve_ms"]["p50"]
    fb.fmmbem_destroy(ctx)
    return out


def laplace_second_kind(args, fb, syn, torch, dev):
    """Second-kind Laplace solve on the 32768-panel sphere (the double layer,
    exterior Neumann problem): du/dn = -(l+1) Y_l^m for the exterior harmonic
    u = Y_l^m / r^(l+1), l = 2; right side -V du/dn by one single-layer FMM
    mat-vec (p = 12, FP64, outside the timing); (1/2 I - K) u = b solved to 1e-6,
    relaxed mixed (p 12 -> 3) against fixed p = 12 FP64, stored near field and
    stored FP64 M2L operators."""
    m = syn.sphere(6)
    Y = syn.ylm_rhs(m, 2, 1)
    sl = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE, fb.params(ncrit=64, p_max=12))
    g = torch.tensor(3.0 * Y, device=dev)  # -du/dn
    b = torch.empty_like(g)
    fb.fmmbem_matvec(sl, 12, fb.FP64, g, b)
    torch.cuda.synchronize()
    fb.fmmbem_destroy(sl)
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE_DL, fb.params(ncrit=64, p_max=12, near_stored=1, m2l_stored=2))
    x = torch.empty_like(b)
    out = {"workload": f"laplace_dl_2nd_kind_sphere{m.n_panels}_exterior_neumann_Y21_tol1e-6",
           "panels": m.n_panels}
    for name, sched in (("relaxed_mixed", fb.schedule(fb.LAPLACE_DL)),
                        ("fixed_p12_fp64", fb.schedule(fb.LAPLACE_DL, rule=fb.FIXED, p_min=12, mixed=0))):
        fb.fmmbem_solve_ctx(ctx, b, TOL, sched, x)  # warm-up
        ts, reps = timed_solves(fb, torch, ctx, b, x, sched, args.cmp_reps)
        err = float(torch.linalg.norm(x - torch.tensor(Y, device=dev)) / np.linalg.norm(Y))
        out[name] = {"solve_ms": summary_ms(ts), **rep_summary(reps), "closed_form_rel_err": err,
                     "p_hist": [int(v) for v in reps[-1]["p_hist"]]}
    out["speedup_relaxed_vs_fixed"] = out["fixed_p12_fp64"]["solve_ms"]["p50"] / out["relaxed_mixed"]["solve_ms"]["p50"]
    fb.fmmbem_destroy(ctx)
    return out


# ------------------------------------------------------------------ serving
def _requests(fb, syn, n_req, rate_hz):
    reqs = syn.request_stream(n_req, rate_hz, 0)
    work = []
    for r in reqs:  # meshes and data before the clock starts
        mesh = r.mesh()
        kernel = fb.LAPLACE if r.kernel == "laplace" else fb.STOKES
        bc = np.ones(mesh.n_panels) if kernel == fb.LAPLACE else np.tile([1.0, 0.0, 0.0], mesh.n_panels)
        work.append((r, mesh, kernel, bc))
    return work


def _serve(fb, work, budget, max_active, saturate=False):
    scheds = {fb.LAPLACE: fb.schedule(fb.LAPLACE), fb.STOKES: fb.schedule(fb.STOKES)}
    srv = fb.fmmbem_server_create(hbm_budget_bytes=budget, max_active=max_active, n_streams=max_active)
    tickets = []
    t0 = time.perf_counter()
    for r, mesh, kernel, bc in work:
        if not saturate:
            dt = r.arrival_s - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
        tickets.append((fb.fmmbem_submit(srv, mesh.xyz, mesh.tri, bc, kernel, TOL, scheds[kernel]), bc.shape[0],
                        kernel, mesh.n_panels))
    infos = []
    for tk, n, kernel, npan in tickets:
        _, info = fb.fmmbem_wait(srv, tk, n)
        infos.append((info, kernel, npan))
    fb.fmmbem_server_destroy(srv)
    lat = np.array([i["finish_s"] - i["arrival_s"] for i, _, _ in infos])
    wait = np.array([i["admit_s"] - i["arrival_s"] for i, _, _ in infos])
    span = max(i["finish_s"] for i, _, _ in infos) - min(i["arrival_s"] for i, _, _ in infos)
    return {"latency_ms": {"p50": 1e3 * pct(lat, 50), "p99": 1e3 * pct(lat, 99), "max": 1e3 * float(lat.max())},
            "queue_wait_ms": {"p50": 1e3 * pct(wait, 50), "p99": 1e3 * pct(wait, 99)},
            "completed_per_s": len(infos) / span,
            "converged": int(sum(int(i["converged"]) for i, _, _ in infos)),
            "peak_device_bytes_request": int(max(i["device_bytes"] for i, _, _ in infos)),
            "unknowns_per_s": sum((3 if k == fb.STOKES else 1) * p for _, k, p in infos) / span}


def serving(args, fb, syn):
    """512 solve requests (Laplace or Stokes on sphere, ellipsoid or RBC
    surfaces of 512 to 32768 panels, tol 1e-6, relaxed mixed schedules)
    through the request loop with an 8 GB admission budget.  The mean solo
    service time T is measured first (one request at a time, the first 48 of
    the stream); Poisson arrivals then run at 0.5, 0.8 and 1.2 / T, and a
    saturation run submits all 512 at once.  Latency = arrival to done."""
    n_req = args.serve_requests
    budget = 8 << 30
    base = _requests(fb, syn, n_req, 1.0)
    # solo service time: each request alone in the loop
    solo = []
    scheds = {fb.LAPLACE: fb.schedule(fb.LAPLACE), fb.STOKES: fb.schedule(fb.STOKES)}
    srv = fb.fmmbem_server_create(hbm_budget_bytes=budget, max_active=1, n_streams=1)
    for r, mesh, kernel, bc in base[:args.serve_calib]:
        tk = fb.fmmbem_submit(srv, mesh.xyz, mesh.tri, bc, kernel, TOL, scheds[kernel])
        _, info = fb.fmmbem_wait(srv, tk, bc.shape[0])
        solo.append(info["finish_s"] - info["arrival_s"])
    fb.fmmbem_server_destroy(srv)
    T = float(np.mean(solo))
    out = {"workload": f"{n_req} requests, Laplace|Stokes on sphere|ellipsoid|RBC, 512-32768 panels, tol 1e-6, "
                       f"8 GB admission budget, 16 slots, 16 streams",
           "solo_service_ms": {"mean": 1e3 * T, "p50": 1e3 * pct(solo, 50), "n": len(solo)}}
    for f in args.serve_loads:
        lam = f / T
        work = [(type(r)(r.ticket, r.arrival_s / lam, r.kernel, r.shape, r.level, r.axes), mesh, k, bc)
                for r, mesh, k, bc in base]
        print(f"bench: serving at {f:g} x 1/T = {lam:.1f} requests/s", file=sys.stderr, flush=True)
        res = _serve(fb, work, budget, 16)
        res["offered_per_s"] = lam
        out[f"load_{f:g}"] = res
    print("bench: serving at saturation", file=sys.stderr, flush=True)
    out["saturation"] = _serve(fb, base, budget, 16, saturate=True)
    return out


# ------------------------------------------------------------------ N_CRIT sweep
def ncrit_sweep(args, fb, syn, torch, dev):
    """Solve time against N_CRIT for both schedules on the Laplace 32768-panel
    sphere (on-the-fly near field) and the 64-cell Stokes case (with the
    headline's M2L, --m2l), and for the cells the mat-vec time per order."""
    out = {"laplace_sphere32768": {}, "stokes_64rbc": {}}
    m = syn.sphere(6)
    b = torch.tensor(syn.ylm_rhs(m, 3, 0), device=dev)
    x = torch.empty_like(b)
    for nc in (16, 32, 64, 128):
        ctx = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE, fb.params(ncrit=nc, p_max=12))
        row = {}
        for name, s in (("relaxed_mixed", fb.schedule(fb.LAPLACE, p_init=12, p_min=3)),
                        ("fixed_p12_fp64", fb.schedule(fb.LAPLACE, rule=fb.FIXED, p_init=12, p_min=12, mixed=0))):
            fb.fmmbem_solve_ctx(ctx, b, TOL, s, x)
            ts, reps = timed_solves(fb, torch, ctx, b, x, s, 5)
            row[name] = summary_ms(ts)["p50"]
        out["laplace_sphere32768"][nc] = row
        print(f"bench: sweep laplace N_CRIT {nc}: {row}", file=sys.stderr, flush=True)
        fb.fmmbem_destroy(ctx)
    m = syn.rbc_scene(64, 4, 0)
    u = torch.tensor(np.tile([1.0, 0.0, 0.0], m.n_panels), device=dev)
    x = torch.empty_like(u)
    for nc in (48, 64, 96, 112, 128, 160, 192, 256, 384):
        ctx = fb.fmmbem_build(m.xyz, m.tri, fb.STOKES, fb.params(ncrit=nc, p_max=16, m2l_stored=M2L_MODES[args.m2l]))
        row = {}
        for name, s in (("relaxed_mixed", fb.schedule(fb.STOKES, p_init=16, p_min=4)),
                        ("fixed_p16_fp64", fb.schedule(fb.STOKES, rule=fb.FIXED, p_init=16, p_min=16, mixed=0))):
            fb.fmmbem_solve_ctx(ctx, u, TOL, s, x)
            ts, reps = timed_solves(fb, torch, ctx, u, x, s, 2)
            row[name] = summary_ms(ts)["p50"]
        # per-order mat-vec times: what a second cut of the tree for some orders would trade
        mv = matvec_times(fb, torch, ctx, u, [(p, fb.FP32) for p in (4, 5, 6, 7, 10, 14)] + [(16, fb.FP64)], 20)
        row["matvec_p50_ms"] = {k: v["p50"] for k, v in mv.items()}
        out["stokes_64rbc"][nc] = row
        print(f"bench: sweep 64 cells N_CRIT {nc}: {row}", file=sys.stderr, flush=True)
        fb.fmmbem_destroy(ctx)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed relaxed solves of the 64-cell case")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--ncrit-relaxed", type=int, default=112)
    ap.add_argument("--ncrit-fixed", type=int, default=192)
    ap.add_argument("--fixed-reps", type=int, default=5, help="fixed-p solves of the 64-cell case (>= 5)")
    ap.add_argument("--m2l", choices=tuple(M2L_MODES), default="rot",
                    help="M2L of the 64-cell case: FP64 operators stored at build, generated per mat-vec, "
                         "or by rotation from p = 7")
    ap.add_argument("--cmp-reps", type=int, default=20, help="solves per schedule of the secondary workloads")
    ap.add_argument("--matvec-reps", type=int, default=100, help="event-timed mat-vecs per order")
    ap.add_argument("--cpu-rows", type=int, default=4096, help="rows of the oracle's sampled mat-vec")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-cpu-sphere", action="store_true", help="skip the oracle's full Laplace mat-vecs")
    ap.add_argument("--timed-only", action="store_true",
                    help="build, warm-up and the timed region only (for profiling the timed kernels)")
    ap.add_argument("--no-extra", action="store_true", help="headline only: no secondary sections")
    ap.add_argument("--laplace-timed-only", action="store_true",
                    help="only the relaxed solves of the 32768-panel Laplace sphere (for profiling them)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-calib", type=int, default=48)
    ap.add_argument("--serve-loads", type=float, nargs="*", default=[0.5, 0.8, 1.2])
    ap.add_argument("--ncrit-sweep", action="store_true", help="only the N_CRIT sweep (one JSON line)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (3 times), to scale HBM counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": a.numel() * 8, "launches": 3}))
        return

    import synthetic as syn
    from paper_1506_05957_amd import fmmbem as fb

    dev = torch.device("cuda:0")
    if args.ncrit_sweep:
        print(json.dumps({"ncrit_sweep": ncrit_sweep(args, fb, syn, torch, dev)}))
        return
    if args.laplace_timed_only:
        print(json.dumps(laplace_timed(args, fb, syn, torch, dev)))
        return

    head = cells_headline(args, fb, syn, torch, dev)
    sections = {}
    sphere_mesh = sphere_x = None
    if not args.timed_only and not args.no_extra:
        for name, fn in (("laplace_sphere2048", laplace_sphere_2048), ("stokes_sphere8192", stokes_sphere_8192),
                         ("laplace_2nd_kind", laplace_second_kind)):
            print(f"bench: {name}", file=sys.stderr, flush=True)
            sections[name] = fn(args, fb, syn, torch, dev)
        print("bench: laplace_sphere32768", file=sys.stderr, flush=True)
        sections["laplace_sphere32768"], sphere_mesh, sphere_x = laplace_sphere_32768(args, fb, syn, torch, dev)
        if not args.no_serving:
            sections["serving"] = serving(args, fb, syn)
    cpu = None
    if not args.timed_only and not args.no_cpu:
        print("bench: CPU oracle", file=sys.stderr, flush=True)
        cpu = cpu_baseline(args, fb, syn, head, sphere_mesh, sphere_x)

    stats = head["stats"]
    rel = head["relaxed"]
    fixed = head.get("fixed")
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * head["t_total"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "stokes_sl_64rbc_131072panels_uniform_flow_relaxed16to4_mixed_tol1e-6",
                   "panels": stats["n_panels"], "unknowns": stats["n_unknowns"], "sources": stats["n_sources"],
                   "cells": 64, "panels_per_cell": 2048, "scene_seed": 0, "mu": 1.0, "theta": 0.5,
                   "ncrit": args.ncrit_relaxed, "restart": 50, "near_field": "on the fly", "m2l": args.m2l},
        "solve_ms": {"relaxed_mixed": rel["solve_ms"], "fixed_p16_fp64": fixed["solve_ms"] if fixed else None},
        "speedup_relaxed_vs_fixed": fixed["solve_ms"]["p50"] / rel["solve_ms"]["p50"] if fixed else None,
        "relaxed_mixed": {k: v for k, v in rel.items() if k != "solve_ms"},
        "fixed_p16_fp64": {k: v for k, v in fixed.items() if k != "solve_ms"} if fixed else None,
        "relaxed_same_tree_as_fixed": head.get("relaxed_same_tree_as_fixed"),
        "force_rel_diff_relaxed_vs_fixed": head.get("force_rel_diff_relaxed_vs_fixed"),
        "matvec_ms": head.get("matvec_ms"),
        "stage_ms_per_solve": head["stage_ms_per_solve"],
        "roofline": head["roofline"],
        "roofline_by_stage": head["roofline_by_stage"],
        "cpu_baseline": cpu,
        "build_s": head["build_s"],
        "tree": {k: stats[k] for k in ("n_boxes", "n_leaves", "n_levels", "n_m2l", "n_p2p", "nnz_correction",
                                       "p2p_interactions", "device_bytes")},
        **sections,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
