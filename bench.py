"""Benchmark: relaxed-order mixed-precision GMRES solves of the Laplace
single-layer BEM system on a 32768-triangle unit sphere, against fixed p.

Workload (synthetic, seeded): octahedron sphere refined to 8*4^6 = 32768 flat
triangles, centroid collocation, 4-point Gauss rule, boundary data
phi = Y_l^m(c/|c|) for l = 0..4 with m drawn from default_rng(0); FMM with
N_CRIT = 64, theta = 0.5; GMRES(50) to a relative residual of 1e-6.
A step is one relaxed solve (p from 12 down to p_min = 3 by the residual,
FP32 P2P/expansions once eps_k >= 1e-5, FP64 Arnoldi), cycling over the five
right-hand sides; inputs are resident in device memory before timing starts.
The line also reports the fixed-p (p = 12, FP64) solve time, the FP64-only
relaxed solve time, mat-vec rates, the per-stage split, the roofline of the
dominant kernel and the oracle's CPU rate on a bounded sample.  Three more
sections, outside the timed region: the second-kind Laplace solve (double
layer, exterior Neumann, 32768 panels), the 64-cell Stokes case (131072
panels, relaxed mixed vs fixed p = 16 FP64, each at its best N_CRIT) and a
512-request serving stream through the request loop (latency p50/p99 from
arrival to done).  The near field of the main workload is stored as a
block-sparse matrix (--near fly evaluates it per mat-vec instead).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]
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
PEAK_FP32_VALU = 157.3e12  # MI355X published FP32 vector peak
PEAK_FP64_VALU = 78.6e12
PEAK_HBM = 8.0e12  # bytes/s


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def ms_pct(a, q):
    """q-th percentile of times a in ms, or None when nothing was timed."""
    return 1e3 * pct(a, q) if len(a) else None


# source regions the HBM counter records were taken on: file, first marker, end marker
COUNTED_SOURCES = {
    "k_p2p<float, false>": [("fmm.hip", "// P2P: one block per work unit", "// ----"), ("tree.hip", "// P2P work units", "}  // namespace")],
    "k_near_spmv<float, false>": [("nearfield.hip", "// y_near = stored near field", "}  // namespace")],
    "k_near_spmv<double, false>": [("nearfield.hip", "// y_near = stored near field", "}  // namespace")],
    "k_m2l_valu<double, 1, 8>": [("fmm.hip", "// The same pass 1 on the vector units", "// Pass 2:")],
    "k_m2l_stored<1>": [("fmm.hip", "// Pass 1 in FP64 from the stored operators",
                         "template <typename R> size_t m2l_mfma_shm")],
    "k_m2l_reduce<double, 1, false>": [("fmm.hip", "// Pass 2: L(T) = sum of Y", "\n}\n")],
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


def kernel_traffic(kernel: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter records
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when there is no
    record or the kernel's source changed since the counters were taken."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*hbm_counters*.md"))):
        try:
            with open(path) as f:
                text = f.read()
            recs = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        except (OSError, IndexError, ValueError):
            continue
        for rec in recs if isinstance(recs, list) else [recs]:
            if rec.get("kernel") != kernel:
                continue
            try:
                if rec.get("source_sha1") != source_sha1(kernel):
                    return None
            except (OSError, ValueError, KeyError):
                return None
            return float(rec["traffic_bytes_per_launch"])
    return None



def stokes_cells(fb, syn, torch, dev, ncrit_relaxed=128, ncrit_fixed=256):
    """64 red-blood-cell surfaces (Evans-Fung, 2048 panels each, 131072 panels, 393216
    unknowns) in uniform flow u = (1, 0, 0): relaxed mixed-precision solve (p 16 -> 4)
    against fixed p = 16 in FP64, both to a relative residual of 1e-6, each at the
    N_CRIT that makes it fastest (as the paper tunes N_CRIT per run)."""
    m = syn.rbc_scene(64, 4, 0)
    u = torch.tensor(np.tile([1.0, 0.0, 0.0], m.n_panels), device=dev)
    x = torch.empty_like(u)
    out = {"workload": "stokes_sl_64rbc_2048panels_uniform_flow_tol1e-6", "panels": m.n_panels,
           "unknowns": 3 * m.n_panels}
    runs = (("relaxed_mixed", fb.schedule(fb.STOKES), ncrit_relaxed),
            ("fixed_p16_fp64", fb.schedule(fb.STOKES, rule=fb.FIXED, p_min=16, mixed=0), ncrit_fixed))
    for name, sched, ncrit in runs:
        t0 = time.perf_counter()
        ctx = fb.fmmbem_build(m.xyz, m.tri, fb.STOKES, fb.params(ncrit=ncrit, p_max=16))
        torch.cuda.synchronize()
        t_build = time.perf_counter() - t0
        fb.fmmbem_solve_ctx(ctx, u, 1e-6, sched, x)  # warm-up
        torch.cuda.synchronize()
        ts = time.perf_counter()
        rep = fb.fmmbem_solve_ctx(ctx, u, 1e-6, sched, x)
        torch.cuda.synchronize()
        out[name] = {"solve_s": time.perf_counter() - ts, "iterations": rep["iterations"],
                     "restarts": rep["restarts"], "rel_res_true": rep["rel_res_true"],
                     "converged": bool(rep["converged"]), "ncrit": ncrit, "build_s": t_build}
        fb.fmmbem_destroy(ctx)
    out["speedup_relaxed_vs_fixed"] = out["fixed_p16_fp64"]["solve_s"] / out["relaxed_mixed"]["solve_s"]
    return out


def laplace_second_kind(fb, syn, torch, dev, level=6, reps=5):
    """Second-kind Laplace solve on the 32768-panel sphere (the double layer,
    exterior Neumann problem): du/dn = -(l+1) Y_l^m for the exterior harmonic
    u = Y_l^m / r^(l+1), l = 2; right side -V du/dn by one single-layer FMM
    mat-vec (p = 12, FP64, outside the timing); (1/2 I - K) u = b solved to 1e-6,
    relaxed mixed (p 12 -> 3) against fixed p = 12 FP64, stored near field and
    stored FP64 M2L operators."""
    m = syn.sphere(level)
    Y = syn.ylm_rhs(m, 2, 1)
    sl = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE, fb.params(ncrit=64, p_max=12))
    g = torch.tensor(3.0 * Y, device=dev)  # -du/dn
    b = torch.empty_like(g)
    fb.fmmbem_matvec(sl, 12, fb.FP64, g, b)
    torch.cuda.synchronize()
    fb.fmmbem_destroy(sl)
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE_DL, fb.params(ncrit=64, p_max=12, near_stored=1, m2l_stored=1))
    x = torch.empty_like(b)
    out = {"workload": f"laplace_dl_2nd_kind_sphere{m.n_panels}_exterior_neumann_Y21_tol1e-6",
           "panels": m.n_panels}
    for name, sched in (("relaxed_mixed", fb.schedule(fb.LAPLACE_DL)),
                        ("fixed_p12_fp64", fb.schedule(fb.LAPLACE_DL, rule=fb.FIXED, p_min=12, mixed=0))):
        fb.fmmbem_solve_ctx(ctx, b, 1e-6, sched, x)  # warm-up
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep = fb.fmmbem_solve_ctx(ctx, b, 1e-6, sched, x)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        err = float(torch.linalg.norm(x - torch.tensor(Y, device=dev)) / np.linalg.norm(Y))
        out[name] = {"solve_ms_p50": 1e3 * pct(ts, 50), "iterations": rep["iterations"],
                     "rel_res_true": rep["rel_res_true"], "closed_form_rel_err": err,
                     "p_hist": [int(v) for v in rep["p_hist"]]}
    out["speedup_relaxed_vs_fixed"] = out["fixed_p12_fp64"]["solve_ms_p50"] / out["relaxed_mixed"]["solve_ms_p50"]
    fb.fmmbem_destroy(ctx)
    return out


def serving(fb, syn, n_req=512, rate_hz=30.0):
    """Serving stream: n_req solve requests with Poisson arrivals at rate_hz, each Laplace or
    Stokes (1/2 each) on a sphere, ellipsoid (axes uniform in [0.5, 2]) or red-blood-cell
    surface of 512 to 32768 panels (log-uniform), tol 1e-6, relaxed mixed schedule; the
    request loop admits them by device-memory footprint.  Latency = arrival to done."""
    reqs = syn.request_stream(n_req, rate_hz, 0)
    work = []
    for r in reqs:  # meshes and data before the clock starts
        mesh = r.mesh()
        kernel = fb.LAPLACE if r.kernel == "laplace" else fb.STOKES
        bc = np.ones(mesh.n_panels) if kernel == fb.LAPLACE else np.tile([1.0, 0.0, 0.0], mesh.n_panels)
        work.append((r, mesh, kernel, bc))
    scheds = {fb.LAPLACE: fb.schedule(fb.LAPLACE), fb.STOKES: fb.schedule(fb.STOKES)}
    srv = fb.fmmbem_server_create(hbm_budget_bytes=64 << 30, max_active=16, n_streams=4)
    tickets = []
    t0 = time.perf_counter()
    for r, mesh, kernel, bc in work:
        dt = r.arrival_s - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append((fb.fmmbem_submit(srv, mesh.xyz, mesh.tri, bc, kernel, 1e-6, scheds[kernel]),
                        bc.shape[0], kernel, mesh.n_panels))
    infos = []
    for tk, n, kernel, npan in tickets:
        _, info = fb.fmmbem_wait(srv, tk, n)
        infos.append((info, kernel, npan))
    fb.fmmbem_server_destroy(srv)
    lat = np.array([i["finish_s"] - i["arrival_s"] for i, _, _ in infos])
    wait = np.array([i["admit_s"] - i["arrival_s"] for i, _, _ in infos])
    span = max(i["finish_s"] for i, _, _ in infos) - min(i["arrival_s"] for i, _, _ in infos)
    return {"workload": f"{n_req} requests, Poisson {rate_hz:g}/s, Laplace|Stokes on sphere|ellipsoid|RBC, "
                        f"512-32768 panels, tol 1e-6",
            "latency_ms": {"p50": 1e3 * pct(lat, 50), "p99": 1e3 * pct(lat, 99), "max": 1e3 * float(lat.max())},
            "queue_wait_ms": {"p50": 1e3 * pct(wait, 50), "p99": 1e3 * pct(wait, 99)},
            "solves_per_s": n_req / span,
            "converged": int(sum(int(i["converged"]) for i, _, _ in infos)),
            "unknowns_per_s": sum((3 if k == fb.STOKES else 1) * p for _, k, p in infos) / span}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--level", type=int, default=6, help="sphere refinement: 8*4^level panels")
    ap.add_argument("--ncrit", type=int, default=64, help="panels per leaf (N_CRIT) of the main workload")
    ap.add_argument("--near", choices=("stored", "fly"), default="stored",
                    help="near field of the main workload: stored block-sparse matrix or evaluated per mat-vec")
    ap.add_argument("--m2l", choices=("stored", "fly"), default="stored",
                    help="FP64 M2L operators of the Laplace workloads: stored at build or generated per mat-vec")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--timed-only", action="store_true",
                    help="warm-up and timed region only: no comparison solves, mat-vec rates, CPU baseline or "
                         "extra cases (for profiling the timed kernels alone)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 64-cell Stokes comparison and the serving stream")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--cells-ncrit", type=int, default=0,
                    help="one N_CRIT for both 64-cell Stokes solves (default: 128 relaxed, 256 fixed)")
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
    mesh = syn.sphere(args.level)
    nt = mesh.n_panels
    orders = syn.ylm_orders(0)
    rhs = [torch.tensor(syn.ylm_rhs(mesh, l, m), device=dev) for l, m in orders]
    prm = fb.params(theta=0.5, ncrit=args.ncrit, p_max=12, near_stored=int(args.near == "stored"),
                    m2l_stored=int(args.m2l == "stored"))
    t0 = time.time()
    ctx = fb.fmmbem_build(mesh.xyz, mesh.tri, fb.LAPLACE, prm)
    torch.cuda.synchronize()
    t_build = time.time() - t0
    stats = fb.fmmbem_get_stats(ctx)
    print(f"bench: built {nt} panels in {t_build:.2f}s: {stats}", file=sys.stderr, flush=True)

    tol = 1e-6
    relaxed = fb.schedule(fb.LAPLACE, rule=fb.RELAX_BF, p_init=12, p_min=3, mixed=1, restart=50)
    relaxed64 = fb.schedule(fb.LAPLACE, rule=fb.RELAX_BF, p_init=12, p_min=3, mixed=0, restart=50)
    fixed = fb.schedule(fb.LAPLACE, rule=fb.FIXED, p_init=12, p_min=12, mixed=0, restart=50)
    x = torch.empty(nt, dtype=torch.float64, device=dev)

    def solve(sched, i):
        return fb.fmmbem_solve_ctx(ctx, rhs[i % len(rhs)], tol, sched, x)

    for i in range(args.warmup):
        solve(relaxed, i)
        solve(fixed, i)
    torch.cuda.synchronize()
    # the dominant kernel stage, from two relaxed solves with every stage timed;
    # the timed region then records events for that stage only (two per
    # mat-vec on its stream), so that it adds little host work to the solves
    fb.fmmbem_set_timing(ctx, True)
    fb.fmmbem_get_timing(ctx, reset=True)
    for i in range(2):
        solve(relaxed, i)
    warm_stage = fb.fmmbem_get_timing(ctx, reset=True)
    dom = max(("p2p_fp32", "p2p_fp64", "m2l_fp32", "m2l_fp64"), key=lambda s: warm_stage[s][0])

    # ---- timed region: K relaxed mixed-precision solves
    fb.fmmbem_set_timing_stages(ctx, [dom])
    fb.fmmbem_get_timing(ctx, reset=True)
    times, iters, matvecs = [], [], 0
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        rep = solve(relaxed, i)
        times.append(time.perf_counter() - ts)
        iters.append(rep["iterations"])
        matvecs += rep["matvecs"]
        assert rep["converged"], rep
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    stage = fb.fmmbem_get_timing(ctx, reset=True)
    fb.fmmbem_set_timing(ctx, False)
    last_p = [int(v) for v in rep["p_hist"]]
    last_prec = [int(v) for v in rep["prec_hist"]]

    # ---- comparison solves (outside the timed region)
    def time_solves(sched, k):
        ts, its = [], []
        for i in range(k):
            torch.cuda.synchronize()
            t = time.perf_counter()
            r = solve(sched, i)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
            its.append(r["iterations"])
        return ts, its

    k_cmp = max(5, min(args.steps, 10))
    if args.timed_only:
        args.no_cpu = args.no_extra = True
        t_fixed = t_rel64 = []
        it_fixed = it_rel64 = [0]
    else:
        t_fixed, it_fixed = time_solves(fixed, k_cmp)
        t_rel64, it_rel64 = time_solves(relaxed64, k_cmp)

    # ---- mat-vec rates
    def matvec_rate(p, prec, reps=50):
        y = torch.empty_like(x)
        fb.fmmbem_matvec(ctx, p, prec, rhs[0], y)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fb.fmmbem_matvec(ctx, p, prec, rhs[0], y)
        torch.cuda.synchronize()
        return reps / (time.perf_counter() - t)

    if args.timed_only:
        mv = {}
    else:
        mv = {"p12_fp64": matvec_rate(12, fb.FP64), "p12_fp32": matvec_rate(12, fb.FP32),
              "p6_fp32": matvec_rate(6, fb.FP32), "p3_fp32": matvec_rate(3, fb.FP32)}

    # ---- roofline of the dominant kernel stage, timed live in the timed region
    t_ms, launches, flops = stage[dom]
    avg_s = t_ms / 1e3 / max(launches, 1)
    stored = args.near == "stored"
    if stored and dom.startswith("p2p"):
        # the stored near field is an HBM-bound product: matrix entries plus the
        # sorted input (read per unit from cache, counted once) and the result
        word = 4 if dom.endswith("fp32") else 8
        nbytes = stats["near_entries"] * word + 3 * 8 * nt
        kname = "k_near_spmv<float, false>" if word == 4 else "k_near_spmv<double, false>"
        achieved = nbytes / avg_s
        roofline = {"bound": "hbm", "kernel": kname, "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9,
                    "unit": "GB/s", "frac": achieved / PEAK_HBM, "traffic": kernel_traffic(kname), "avg_launch_us": avg_s * 1e6,
                    "launches": launches, "bytes_per_launch": nbytes}
    elif dom == "m2l_fp64" and stats["m2l_op_bytes"] > 0:
        # M2L pass 1 from stored operators: each translation's operator streams
        # from HBM once (order 12 = p_max: all of it), plus the multipoles read
        # and the per-pair results written
        nc = 91
        nbytes = stats["m2l_op_bytes"] + stats["n_boxes"] * 2 * nc * 8 + stats["n_m2l"] * 2 * nc * 8
        kname = "k_m2l_stored<1>"
        achieved = nbytes / avg_s
        roofline = {"bound": "hbm", "kernel": kname, "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9,
                    "unit": "GB/s", "frac": achieved / PEAK_HBM, "traffic": kernel_traffic(kname),
                    "avg_launch_us": avg_s * 1e6, "launches": launches, "bytes_per_launch": nbytes,
                    "flops_per_launch": flops / max(launches, 1),
                    "fp64_tflops": flops / max(launches, 1) / avg_s / 1e12}
    else:
        achieved = flops / max(launches, 1) / avg_s
        peak = PEAK_FP32_VALU if dom.endswith("fp32") else PEAK_FP64_VALU
        kname = {"p2p_fp32": "k_p2p<float, false>", "p2p_fp64": "k_p2p<double, false>",
                 "m2l_fp32": "k_m2l_mfma<float, 1>", "m2l_fp64": "k_m2l_valu<double, 1, 8>"}[dom]
        roofline = {"bound": "alu", "kernel": kname, "achieved": achieved / 1e12, "peak": peak / 1e12,
                    "unit": "TFLOP/s", "frac": achieved / peak, "traffic": kernel_traffic(kname),
                    "avg_launch_us": avg_s * 1e6, "launches": launches,
                    "flops_per_launch": flops / max(launches, 1)}

    stage_split = {k: {"ms": round(v[0], 3), "launches": v[1]} for k, v in stage.items() if v[1]}

    # ---- CPU oracle on a bounded sample
    cpu = None
    if not args.no_cpu:
        import oracle
        rng = np.random.default_rng(0)
        nrows = 1024
        rows = np.sort(rng.choice(nt, nrows, replace=False))
        xv = rhs[0].cpu().numpy()
        ts = time.perf_counter()
        oracle.matvec(oracle.LAPLACE, mesh.xyz, mesh.tri, xv, rows=rows)
        t_rows = time.perf_counter() - ts
        t_mv = t_rows * nt / nrows
        n_mv = int(np.mean(it_fixed)) + 1
        t_solve_cpu = t_mv * n_mv
        cpu = {"value": 1.0 / t_solve_cpu, "unit": "solves/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"dense FP64 oracle mat-vec on {nrows} of {nt} rows ({t_rows:.2f}s), scaled to a full "
                         f"mat-vec ({t_mv:.1f}s) times {n_mv} mat-vecs (fixed-p iterations + true residual)",
               "matvec_s": t_mv}

    cells = serve = second = None
    if not args.no_extra:
        print("bench: second-kind Laplace case", file=sys.stderr, flush=True)
        second = laplace_second_kind(fb, syn, torch, dev)
        print("bench: 64-cell Stokes case", file=sys.stderr, flush=True)
        if args.cells_ncrit:
            cells = stokes_cells(fb, syn, torch, dev, args.cells_ncrit, args.cells_ncrit)
        else:
            cells = stokes_cells(fb, syn, torch, dev)
        if not args.no_serving:
            print("bench: serving stream", file=sys.stderr, flush=True)
            serve = serving(fb, syn)

    ms = 1e3 * t_total / args.steps
    out = {
        "metric": METRIC,
        "value": args.steps / t_total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "laplace_sl_sphere32768_ylm_relaxed12to3_tol1e-6", "panels": nt,
                   "rhs": [f"Y_{l}^{m}" for l, m in orders], "ncrit": args.ncrit, "theta": 0.5, "restart": 50,
                   "near_field": args.near, "m2l_fp64": args.m2l},
        "solve_ms": {"relaxed_mixed_p50": 1e3 * pct(times, 50), "relaxed_mixed_p99": 1e3 * pct(times, 99),
                     "relaxed_fp64_p50": ms_pct(t_rel64, 50), "relaxed_fp64_p99": ms_pct(t_rel64, 99),
                     "fixed_p12_fp64_p50": ms_pct(t_fixed, 50), "fixed_p12_fp64_p99": ms_pct(t_fixed, 99)},
        "speedup_relaxed_vs_fixed": None if args.timed_only else pct(t_fixed, 50) / pct(times, 50),
        "iterations": {"relaxed_mixed": float(np.mean(iters)), "relaxed_fp64": float(np.mean(it_rel64)),
                       "fixed": float(np.mean(it_fixed))},
        "matvec_per_s": {"in_relaxed_solves": matvecs / t_total, **mv},
        "p2p_interactions_per_matvec": stats["p2p_interactions"],
        "p2p_interactions_per_s_fp32": stats["p2p_interactions"] * mv["p3_fp32"] if mv else None,
        "p_history_last": last_p, "prec_history_last": last_prec,
        "stage_ms": stage_split,
        "stage_ms_warmup_all_stages": {k: {"ms": round(v[0], 3), "launches": v[1]}
                                       for k, v in warm_stage.items() if v[1]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "laplace_2nd_kind": second,
        "stokes_64cells": cells,
        "serving": serve,
        "build_s": t_build,
        "tree": {k: stats[k] for k in ("n_boxes", "n_leaves", "n_levels", "n_m2l", "n_p2p", "nnz_correction",
                                       "n_translations", "m2l_op_bytes", "near_entries", "device_bytes")},
    }
    print(json.dumps(out))
    fb.fmmbem_destroy(ctx)


if __name__ == "__main__":
    main()
