"""The allocation-free solve (fmmbem_solve_ctx_static) against the solve that
allocates its Krylov workspace (fmmbem_solve_ctx), through the C-ABI.

The two run the same kernels on the same inputs, so their solutions and
reports are equal bit for bit.  Two calls in a row, the second on a smaller
problem, show that the shared static workspace carries nothing from one call
to the next; the size limits are rejected on the host before any work."""
import numpy as np
import pytest
import torch

import synthetic as syn
from gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu


def _pair(fb, mesh, kernel, b, sched, tol):
    ctx = fb.fmmbem_build(mesh.xyz, mesh.tri, kernel, fb.params(ncrit=64, p_max=sched.p_init))
    bd = to_dev(b)
    xa = torch.empty_like(bd)
    xs = torch.empty_like(bd)
    xs.fill_(np.nan)  # whatever the output held before must not matter
    ra = fb.fmmbem_solve_ctx(ctx, bd, tol, sched, xa)
    rs = fb.fmmbem_solve_ctx_static(ctx, bd, tol, sched, xs)
    torch.cuda.synchronize()
    fb.fmmbem_destroy(ctx)
    return xa.cpu().numpy(), ra, xs.cpu().numpy(), rs


def test_static_solve_equals_allocating_solve():
    from paper_1506_05957_amd import fmmbem as fb
    # first call: Stokes on 8 cells x 512 panels (12288 unknowns); second: a
    # smaller Laplace sphere (2048 unknowns) in the same static workspace
    cases = [("stokes cells8x512", syn.rbc_scene(8, 3, 1), fb.STOKES,
              lambda m: np.tile([1.0, 0.0, 0.0], m.n_panels), fb.schedule(fb.STOKES, p_init=16, p_min=4)),
             ("laplace sphere2048", syn.sphere(4), fb.LAPLACE, lambda m: syn.ylm_rhs(m, 3, 0),
              fb.schedule(fb.LAPLACE, p_init=12, p_min=3))]
    for name, mesh, kernel, rhs, sched in cases:
        announce(f"no-alloc solve: {name}")
        xa, ra, xs, rs = _pair(fb, mesh, kernel, rhs(mesh), sched, 1e-6)
        announce(f"  it={ra['iterations']}/{rs['iterations']} true={ra['rel_res_true']:.2e}/{rs['rel_res_true']:.2e}")
        assert ra["converged"] and rs["converged"]
        assert rs["iterations"] == ra["iterations"] and rs["matvecs"] == ra["matvecs"]
        assert rs["rel_res_true"] == ra["rel_res_true"]
        assert np.array_equal(rs["p_hist"], ra["p_hist"]) and np.array_equal(rs["prec_hist"], ra["prec_hist"])
        assert np.array_equal(xs, xa), np.max(np.abs(xs - xa))


def test_static_solve_limits():
    from paper_1506_05957_amd import fmmbem as fb
    m = syn.sphere(3)
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE, fb.params(ncrit=64, p_max=12))
    bd = to_dev(np.ones(m.n_panels))
    xd = torch.empty_like(bd)
    with pytest.raises(fb.FmmbemError) as e:
        fb.fmmbem_solve_ctx_static(ctx, bd, 1e-6, fb.schedule(fb.LAPLACE, restart=65), xd)
    assert e.value.code == fb.EINVAL
    fb.fmmbem_set_timing(ctx, True)
    with pytest.raises(fb.FmmbemError) as e:
        fb.fmmbem_solve_ctx_static(ctx, bd, 1e-6, fb.schedule(fb.LAPLACE), xd)
    assert e.value.code == fb.EINVAL
    fb.fmmbem_set_timing(ctx, False)
    fb.fmmbem_destroy(ctx)
    # GMRES(64) on 131072 unknowns needs 67 x 131072 x 8 B > 64 MiB
    big = syn.sphere(7)
    ctx = fb.fmmbem_build(big.xyz, big.tri, fb.LAPLACE, fb.params(ncrit=64, p_max=3))
    bd = to_dev(np.ones(big.n_panels))
    xd = torch.empty_like(bd)
    with pytest.raises(fb.FmmbemError) as e:
        fb.fmmbem_solve_ctx_static(ctx, bd, 1e-6, fb.schedule(fb.LAPLACE, p_init=3, p_min=3, restart=64), xd)
    assert e.value.code == fb.EINVAL and "workspace" in fb.fmmbem_last_error()
    fb.fmmbem_destroy(ctx)
