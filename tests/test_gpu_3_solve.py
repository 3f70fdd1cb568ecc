"""GMRES solves on the GPU against the oracle's dense GMRES solution.

Reading of "solution within 1e-5 of the FP64 oracle": GMRES stopped at a
relative residual tol leaves a solution error up to cond * tol (3e-5 to 6e-5
here at tol = 1e-6, for fixed and relaxed p alike), so parity is measured at
tol = 1e-8 against the oracle converged to 1e-11, where the stopping error is
below the bar.  At the bench tolerance 1e-6 the tests check the true residual
and that relaxation does not move the solution further from the oracle than
the stopping error itself.

Stokes: the first-kind single layer maps the normal field of each closed
body to (nearly) zero, so a traction is fixed only up to one multiple of the
normal per body, which GMRES picks along its own Krylov path.  Stokes
solutions are therefore compared after removing, body by body, their
area-weighted normal component, and through the force on each body (which the
normal field does not change).
"""
import numpy as np
import pytest
import torch

import synthetic as syn
from gpu_util import MESHES, announce, rel_l2, to_dev

pytestmark = pytest.mark.gpu

RULES = [(0, 0), (2, 0), (2, 1)]  # (rule, mixed): fixed FP64, relaxed FP64, relaxed mixed


def solve(fb, ctx, b, tol, sched):
    bd = to_dev(b)
    xd = torch.empty_like(bd)
    rep = fb.fmmbem_solve_ctx(ctx, bd, tol, sched, xd)
    torch.cuda.synchronize()
    return xd.cpu().numpy(), rep


def describe(rep, x, xo):
    return (f"  it={rep['iterations']} p={[int(v) for v in rep['p_hist']]} "
            f"prec={[int(v) for v in rep['prec_hist']]} true={rep['rel_res_true']:.1e} err={rel_l2(x, xo):.1e}")


def bodies_of(name, n_panels):
    if name.startswith("cells"):
        k = int(name[5:].split("x")[0])
        return [range(i * (n_panels // k), (i + 1) * (n_panels // k)) for i in range(k)]
    return [range(n_panels)]


def strip_normal(orc, m, t, bodies):
    """t minus, per body, its area-weighted normal component."""
    _, S, nrm = orc.panels(m.xyz, m.tri)
    t = t.reshape(-1, 3).copy()
    for b in bodies:
        idx = np.fromiter(b, dtype=np.int64)
        a = np.sum(np.einsum("ij,ij->i", t[idx], nrm[idx]) * S[idx]) / np.sum(S[idx])
        t[idx] -= a * nrm[idx]
    return t.reshape(-1)


def body_forces(orc, m, t, bodies):
    _, S, _ = orc.panels(m.xyz, m.tri)
    t = t.reshape(-1, 3)
    return np.array([np.sum(t[np.fromiter(b, dtype=np.int64)] * S[np.fromiter(b, dtype=np.int64), None], axis=0)
                     for b in bodies])


def compare(orc, kernel, mesh_name, m, x, xo):
    """relative error of x against the oracle solution, null-space free for Stokes"""
    if kernel == 0:
        return rel_l2(x, xo)
    bodies = bodies_of(mesh_name, m.n_panels)
    e = rel_l2(strip_normal(orc, m, x, bodies), strip_normal(orc, m, xo, bodies))
    Fo = body_forces(orc, m, xo, bodies)
    eF = float(np.max(np.abs(body_forces(orc, m, x, bodies) - Fo)) / np.max(np.abs(Fo)))
    return max(e, eF)


CASES = {
    "laplace_sphere_one": (0, "sphere2048", lambda m: np.ones(m.n_panels), 12, 3),
    "laplace_sphere_ylm": (0, "sphere2048", lambda m: syn.ylm_rhs(m, 3, 0), 12, 3),
    "laplace_rbc_ylm": (0, "rbc2048", lambda m: syn.ylm_rhs(m, 2, 1), 12, 3),
    "stokes_sphere_u": (1, "sphere2048", lambda m: np.tile([1.0, 0.0, 0.0], m.n_panels), 16, 4),
    "stokes_cells_u": (1, "cells8x512", lambda m: np.tile([1.0, 0.0, 0.0], m.n_panels), 16, 4),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("rule,mixed", RULES)
def test_solve_parity_tight(orc, case, rule, mixed):
    from paper_1506_05957_amd import fmmbem as fb
    kernel, mesh_name, rhs, p_init, p_min = CASES[case]
    announce(f"solve parity {case} rule={rule} mixed={mixed} tol=1e-8")
    m = MESHES[mesh_name]()
    b = rhs(m)
    xo = orc.solve(kernel, m.xyz, m.tri, b, tol=1e-11)[0]
    ctx = fb.fmmbem_build(m.xyz, m.tri, kernel, fb.params(ncrit=64, p_max=p_init))
    x, rep = solve(fb, ctx, b, 1e-8, fb.schedule(kernel, rule=rule, mixed=mixed, p_init=p_init, p_min=p_min))
    err = compare(orc, kernel, mesh_name, m, x, xo)
    announce(describe(rep, x, xo) + f" cmp={err:.1e}")
    assert rep["converged"]
    assert rep["rel_res_true"] <= 1e-7
    assert err <= 1e-5
    if rule == 0:
        assert set(int(v) for v in rep["p_hist"]) == {p_init}
        assert set(int(v) for v in rep["prec_hist"]) == {0}
    else:
        assert int(rep["p_hist"][0]) == p_init and int(rep["p_hist"][-1]) < p_init
    fb.fmmbem_destroy(ctx)


@pytest.mark.parametrize("case", ["laplace_sphere_ylm", "stokes_cells_u"])
def test_solve_parity_stored_near_field(orc, case):
    """Relaxed mixed solve with the near field stored as a block-sparse matrix
    (the paper's configuration): the same parity bar as on the fly."""
    from paper_1506_05957_amd import fmmbem as fb
    kernel, mesh_name, rhs, p_init, p_min = CASES[case]
    announce(f"solve parity {case} stored near field tol=1e-8")
    m = MESHES[mesh_name]()
    b = rhs(m)
    xo = orc.solve(kernel, m.xyz, m.tri, b, tol=1e-11)[0]
    ctx = fb.fmmbem_build(m.xyz, m.tri, kernel, fb.params(ncrit=64, p_max=p_init, near_stored=1))
    st = fb.fmmbem_get_stats(ctx)
    assert 4 * st["near_entries"] == st["p2p_interactions"]
    x, rep = solve(fb, ctx, b, 1e-8, fb.schedule(kernel, p_init=p_init, p_min=p_min))
    err = compare(orc, kernel, mesh_name, m, x, xo)
    announce(describe(rep, x, xo) + f" cmp={err:.1e}")
    assert rep["converged"] and rep["rel_res_true"] <= 1e-7
    assert err <= 1e-5
    fb.fmmbem_destroy(ctx)


def test_solve_restarts_with_prefetch(orc):
    """GMRES(6) with the relaxed mixed schedule on the bench configuration
    (stored near field and M2L operators): several restarts, each resuming the
    schedule from the true residual, with the next mat-vec's charges (which
    also normalise the Arnoldi vector), upward pass and near field started
    ahead inside every cycle, and |b| read with the first column; parity with
    the oracle at tol 1e-8, the same bits on a second solve, and a zero
    right-hand side right after it converging at once to x = 0."""
    from paper_1506_05957_amd import fmmbem as fb
    announce("restarted relaxed solve, rbc2048, GMRES(6), stored near field and M2L operators")
    m = MESHES["rbc2048"]()
    b = syn.ylm_rhs(m, 2, 1)
    xo = orc.solve(0, m.xyz, m.tri, b, tol=1e-11)[0]
    ctx = fb.fmmbem_build(m.xyz, m.tri, 0, fb.params(ncrit=64, p_max=12, near_stored=1, m2l_stored=1))
    sched = fb.schedule(0, restart=6)
    x, rep = solve(fb, ctx, b, 1e-8, sched)
    announce(describe(rep, x, xo) + f" restarts={rep['restarts']}")
    assert rep["converged"] and rep["restarts"] >= 2 and rep["rel_res_true"] <= 1e-7
    assert rel_l2(x, xo) <= 1e-5
    x2, rep2 = solve(fb, ctx, b, 1e-8, sched)
    assert np.array_equal(x, x2) and rep2["iterations"] == rep["iterations"]
    z, repz = solve(fb, ctx, np.zeros_like(b), 1e-6, sched)
    assert repz["converged"] and repz["iterations"] == 0 and not z.any()
    fb.fmmbem_destroy(ctx)


@pytest.mark.parametrize("case", ["laplace_sphere_one", "stokes_sphere_u"])
def test_solve_bench_tolerance(orc, case):
    from paper_1506_05957_amd import fmmbem as fb
    kernel, mesh_name, rhs, p_init, p_min = CASES[case]
    announce(f"solve at tol 1e-6 {case}")
    m = MESHES[mesh_name]()
    b = rhs(m)
    xo = orc.solve(kernel, m.xyz, m.tri, b, tol=1e-11)[0]
    ctx = fb.fmmbem_build(m.xyz, m.tri, kernel, fb.params(ncrit=64, p_max=p_init))
    xf, rf = solve(fb, ctx, b, 1e-6, fb.schedule(kernel, rule=0, mixed=0, p_init=p_init, p_min=p_init))
    xr, rr = solve(fb, ctx, b, 1e-6, fb.schedule(kernel, p_init=p_init, p_min=p_min))
    announce(describe(rf, xf, xo))
    announce(describe(rr, xr, xo))
    assert rf["converged"] and rr["converged"]
    assert rr["rel_res_true"] <= 1.5e-6
    ef, er = compare(orc, kernel, mesh_name, m, xf, xo), compare(orc, kernel, mesh_name, m, xr, xo)
    announce(f"  fixed {ef:.1e} relaxed {er:.1e}")
    assert er <= 2 * ef + 1e-5
    if kernel == 1:
        F, _ = orc.force_torque(m.xyz, m.tri, xr)
        assert abs(F[0] + 6 * np.pi) / (6 * np.pi) < 5e-3
    fb.fmmbem_destroy(ctx)


def test_one_shot_solve_and_errors(orc):
    from paper_1506_05957_amd import fmmbem as fb
    announce("one-shot fmmbem_solve + argument errors")
    m = MESHES["sphere512"]()
    b = np.ones(m.n_panels)
    x, rep = fb.fmmbem_solve(m.xyz, m.tri, b, fb.LAPLACE, 1e-8, fb.schedule(fb.LAPLACE))
    xo = orc.solve(orc.LAPLACE, m.xyz, m.tri, b, tol=1e-11)[0]
    assert rep["converged"] and rel_l2(x, xo) < 1e-5
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE, fb.params(p_max=12))
    bd = to_dev(b); xd = torch.empty_like(bd)
    for kw in (dict(p_min=13), dict(p_init=13), dict(restart=0)):
        with pytest.raises(fb.FmmbemError) as e:
            fb.fmmbem_solve_ctx(ctx, bd, 1e-6, fb.schedule(fb.LAPLACE, **kw), xd)
        assert e.value.code == fb.EINVAL
    with pytest.raises(fb.FmmbemError):
        fb.fmmbem_solve_ctx(ctx, bd, 0.0, fb.schedule(fb.LAPLACE), xd)
    # p_min = 1 with a 3-iteration cap does not converge: ENOCONV, x and report still filled
    rep = fb.fmmbem_solve_ctx(ctx, bd, 1e-12, fb.schedule(fb.LAPLACE, p_min=1, max_iter=3), xd)
    assert rep["status"] == fb.ENOCONV and rep["iterations"] == 3 and not rep["converged"]
    assert np.isfinite(xd.cpu().numpy()).all()
    # zero right-hand side converges at once to x = 0
    z = torch.zeros_like(bd)
    rep = fb.fmmbem_solve_ctx(ctx, z, 1e-6, fb.schedule(fb.LAPLACE), xd)
    assert rep["converged"] and rep["iterations"] == 0 and float(xd.abs().max()) == 0.0
    fb.fmmbem_destroy(ctx)
