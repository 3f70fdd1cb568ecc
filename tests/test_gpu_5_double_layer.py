"""Laplace double layer, second kind: the GPU operator 1/2 I - K against
the oracle's dense operator, the error of the expansions against p, and the
exterior Neumann solve against the oracle and the closed form on the sphere."""
import numpy as np
import pytest
import torch

import synthetic as syn
from gpu_util import MESHES, announce, rel_l2, to_dev

pytestmark = pytest.mark.gpu


def matvec(fb, ctx, p, prec, x):
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    fb.fmmbem_matvec(ctx, p, prec, xd, yd)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


@pytest.mark.parametrize("near_stored", [0, 1])
@pytest.mark.parametrize("name", ["sphere512", "rbc2048"])
def test_dl_all_p2p_equals_dense(orc, name, near_stored):
    from paper_1506_05957_amd import fmmbem as fb
    announce(f"double layer all-P2P {name} near_stored={near_stored}")
    m = MESHES[name]()
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE_DL, fb.params(theta=1e-6, ncrit=32, near_stored=near_stored))
    assert fb.fmmbem_get_stats(ctx)["n_m2l"] == 0
    x = syn.random_vector(m.n_panels, 31)
    yr = orc.matvec(orc.LAPLACE_DL, m.xyz, m.tri, x)
    assert rel_l2(matvec(fb, ctx, 4, fb.FP64, x), yr) < 1e-12
    assert rel_l2(matvec(fb, ctx, 4, fb.FP32, x), yr) < 2e-6
    fb.fmmbem_destroy(ctx)


@pytest.mark.parametrize("name", ["sphere2048", "rbc2048"])
def test_dl_error_falls_with_p(orc, name):
    from paper_1506_05957_amd import fmmbem as fb
    announce(f"double layer error vs p {name}")
    m = MESHES[name]()
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE_DL, fb.params(ncrit=32, p_max=16))
    assert fb.fmmbem_get_stats(ctx)["n_m2l"] > 0
    x = syn.random_vector(m.n_panels, 32)
    yr = orc.matvec(orc.LAPLACE_DL, m.xyz, m.tri, x)
    errs = {}
    for p in (2, 4, 6, 8, 12, 16):
        errs[p] = rel_l2(matvec(fb, ctx, p, fb.FP64, x), yr)
    announce("  " + " ".join(f"p{p}={e:.1e}" for p, e in errs.items()))
    assert errs[6] <= 1e-3 and errs[12] <= 1e-6 and errs[16] <= 1e-6
    assert errs[2] > errs[4] > errs[6] > errs[8] > errs[12]
    e32 = rel_l2(matvec(fb, ctx, 6, fb.FP32, x), yr)
    assert e32 <= 1e-3
    fb.fmmbem_destroy(ctx)


@pytest.mark.parametrize("rule,mixed", [(0, 0), (2, 1)])
def test_dl_exterior_neumann_parity(orc, rule, mixed):
    from paper_1506_05957_amd import fmmbem as fb
    announce(f"double layer exterior Neumann solve rule={rule} mixed={mixed}")
    m = MESHES["sphere2048"]()
    l, mm = 2, 1
    Y = syn.ylm_rhs(m, l, mm)
    b = -orc.matvec(orc.LAPLACE, m.xyz, m.tri, -(l + 1) * Y)  # -V du/dn, u = Y / r^(l+1)
    xo = orc.solve(orc.LAPLACE_DL, m.xyz, m.tri, b, tol=1e-11)[0]
    ctx = fb.fmmbem_build(m.xyz, m.tri, fb.LAPLACE_DL, fb.params(ncrit=64, p_max=12))
    bd = to_dev(b)
    xd = torch.empty_like(bd)
    rep = fb.fmmbem_solve_ctx(ctx, bd, 1e-8, fb.schedule(fb.LAPLACE_DL, rule=rule, mixed=mixed, p_init=12, p_min=3),
                              xd)
    x = xd.cpu().numpy()
    err = rel_l2(x, xo)
    ecl = rel_l2(x, Y)
    announce(f"  it={rep['iterations']} true={rep['rel_res_true']:.1e} vs oracle {err:.1e} vs closed form {ecl:.1e}")
    assert rep["converged"] and rep["rel_res_true"] <= 1e-7
    assert rep["iterations"] <= 15
    assert err <= 1e-5
    assert ecl <= 1e-2
    fb.fmmbem_destroy(ctx)
