"""Red-blood-cell studies of Sec. 3.3 through the same GPU path.

  python -m paper_1506_05957_amd.studies [--out FILE]

Prints one JSON object with three studies, all Stokes single layer, uniform
flow u = (1, 0, 0), mu = 1e-3, one Evans-Fung cell (Eq. 21) of 8 um diameter
or several copies in random non-overlapping positions and orientations:

  richardson  drag f_x = sum_j t_x,j S_j of one cell at N = 512, 2048, 8192
              and 32768 panels (tol 1e-6, relaxed mixed schedule p 16 -> 4),
              the extrapolated value (f1 f3 - f2^2) / (f1 - 2 f2 + f3) and the
              observed order ln((f2 - f1)/(f3 - f2)) / ln 4 from the first three;
  iterations  GMRES iterations to 1e-5 at fixed p = 16 for one cell,
              N = 128 ... 32768 (the paper reports 18 rising to 39);
  cells       iterations to 1e-5 (p = 16, p_min = 5, relaxed) for 2, 4 and 8
              cells of 2048, 8192 and 32768 panels each (the paper: 45-65).

The drag is a plain post-processing of the tractions (panel areas from the
mesh); every solve runs in libfmmbem.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MU = 1e-3


def panel_areas(xyz, tri):
    a = xyz[tri[:, 1]] - xyz[tri[:, 0]]
    b = xyz[tri[:, 2]] - xyz[tri[:, 0]]
    return 0.5 * np.linalg.norm(np.cross(a, b), axis=1)


def solve_cell(fb, torch, mesh, tol, sched, ncrit=64):
    ctx = fb.fmmbem_build(mesh.xyz, mesh.tri, fb.STOKES, fb.params(ncrit=ncrit, p_max=16, mu=MU))
    u = torch.tensor(np.tile([1.0, 0.0, 0.0], mesh.n_panels), device="cuda:0")
    t = torch.empty_like(u)
    t0 = time.perf_counter()
    rep = fb.fmmbem_solve_ctx(ctx, u, tol, sched, t)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fb.fmmbem_destroy(ctx)
    return t.cpu().numpy().reshape(-1, 3), rep, dt


def richardson(fb, syn, torch, levels=(3, 4, 5, 6)):
    relaxed = fb.schedule(fb.STOKES)
    rows = []
    for level in levels:
        m = syn.rbc(level)
        t, rep, dt = solve_cell(fb, torch, m, 1e-6, relaxed)
        fx = float(np.sum(t[:, 0] * panel_areas(m.xyz, m.tri)))
        rows.append({"panels": m.n_panels, "f_x": fx, "iterations": rep["iterations"], "solve_s": dt,
                     "converged": bool(rep["converged"])})
    f1, f2, f3 = (r["f_x"] for r in rows[:3])
    den = f1 - 2 * f2 + f3
    fbar = (f1 * f3 - f2 * f2) / den if den != 0 else float("nan")
    ratio = (f2 - f1) / (f3 - f2) if f3 != f2 else float("nan")
    order = math.log(ratio) / math.log(4.0) if ratio > 0 else float("nan")
    for r in rows:
        r["error_vs_extrapolated"] = abs(r["f_x"] - fbar) / abs(fbar) if math.isfinite(fbar) else None
    return {"meshes": rows, "f_extrapolated": fbar, "observed_order": order,
            "paper": {"f_x": {"512": -0.057, "2048": -0.070, "8192": -0.077}, "observed_order": 0.52}}


def iterations_vs_n(fb, syn, torch, levels=(2, 3, 4, 5, 6)):
    fixed = fb.schedule(fb.STOKES, rule=fb.FIXED, p_min=16, mixed=0)
    out = []
    for level in levels:
        m = syn.rbc(level)
        _, rep, dt = solve_cell(fb, torch, m, 1e-5, fixed)
        out.append({"panels": m.n_panels, "iterations": rep["iterations"], "solve_s": dt,
                    "converged": bool(rep["converged"])})
    return {"runs": out, "paper": "18 iterations at N = 128 rising to 39 at 8192, about the same beyond"}


def multi_cell(fb, syn, torch, cells=(2, 4, 8), levels=(4, 5, 6)):
    sched = fb.schedule(fb.STOKES, p_init=16, p_min=5)
    out = []
    for n_cells in cells:
        for level in levels:
            m = syn.rbc_scene(n_cells, level, 0)
            _, rep, dt = solve_cell(fb, torch, m, 1e-5, sched)
            out.append({"cells": n_cells, "panels_per_cell": m.n_panels // n_cells, "iterations": rep["iterations"],
                        "solve_s": dt, "converged": bool(rep["converged"])})
    return {"runs": out, "paper": "45 to 65 iterations, rising with the number of cells"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="also write the JSON to this file")
    args = ap.parse_args()
    import torch

    import synthetic as syn
    from paper_1506_05957_amd import fmmbem as fb

    res = {"mu": MU, "u": [1.0, 0.0, 0.0]}
    for name, fn in (("richardson", richardson), ("iterations", iterations_vs_n), ("cells", multi_cell)):
        print(f"studies: {name}", file=sys.stderr, flush=True)
        res[name] = fn(fb, syn, torch)
    text = json.dumps(res)
    print(text)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text + "\n")


if __name__ == "__main__":
    main()
