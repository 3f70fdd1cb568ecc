"""Pins for the oracle's Laplace double-layer operator, second kind (Sec. 2.1,
Eq. 5 and 11), written for the exterior Neumann problem with outward normals:
(1/2 I - K) u = -V du/dn, K u = int u dG/dn_y, G = 1/(4 pi r).

Closed forms on the unit sphere (continuous operators):
  * Gauss's identity: int_S dG/dn_y dS = -1/2 at a point of S, so (1/2 - K) 1 = 1.
  * Exterior harmonic u = Y_l^m / r^(l+1): on r = 1, u = Y, du/dn = -(l+1) Y and
    K Y = -Y / (2 (2l+1)), so (1/2 - K) Y = (l+1)/(2l+1) Y.
  * The exterior Neumann solve with du/dn = -(l+1) Y returns u = Y, its right
    side -V du/dn formed with the single-layer oracle.
The flat-panel discretisation error must be small and must fall under refinement.
Entry accuracy: far entries against an independent high-order integral; the
target's own panel gives 0 (the kernel vanishes in the panel's plane).
"""
import numpy as np
import pytest

import synthetic as syn


def high_order_dl_integral(v0, v1, v2, nrm, x, n=40):
    """int_T n . (x - y) / |x - y|^3 dA with an n x n collapsed Gauss-Legendre rule."""
    g, w = np.polynomial.legendre.leggauss(n)
    s = 0.5 * (g + 1)
    ws = 0.5 * w
    S, Tt = np.meshgrid(s, s, indexing="ij")
    W = np.outer(ws, ws) * S
    l1 = S * (1 - Tt)
    l2 = S * Tt
    l0 = 1 - S
    Y = l0[..., None] * v0 + l1[..., None] * v1 + l2[..., None] * v2
    d = x - Y
    r = np.linalg.norm(d, axis=-1)
    area2 = np.linalg.norm(np.cross(v1 - v0, v2 - v0))
    return np.sum(W * (d @ nrm) / r ** 3) * area2


def test_gauss_identity(orc):
    errs = []
    for lev in (2, 3, 4):
        m = syn.sphere(lev)
        y = orc.matvec(orc.LAPLACE_DL, m.xyz, m.tri, np.ones(m.n_panels))
        errs.append(np.max(np.abs(y - 1.0)))
    # calibrated on this oracle: 4.3e-4, 1.5e-4, 6.7e-5
    assert errs[-1] < 1e-4
    assert errs[0] > errs[1] > errs[2]


@pytest.mark.parametrize("l,m", [(1, 0), (2, 1), (3, -2)])
def test_sphere_eigenvalues(orc, l, m):
    errs = []
    for lev in (2, 3, 4):
        mesh = syn.sphere(lev)
        Y = syn.ylm_rhs(mesh, l, m)
        y = orc.matvec(orc.LAPLACE_DL, mesh.xyz, mesh.tri, Y)
        lam = (l + 1) / (2 * l + 1)
        errs.append(np.linalg.norm(y - lam * Y) / np.linalg.norm(lam * Y))
    # second order in h: each refinement divides the error by about 4
    assert errs[-1] < 2e-3 * (l + 1)
    assert errs[0] > 3 * errs[1] > 9 * errs[2]


def test_self_entry_is_zero_and_far_entries(orc):
    m = syn.sphere(3)
    c, S, nrm = orc.panels(m.xyz, m.tri)
    assert orc.laplace_dl_entry(m.xyz, m.tri, 7, 7) == 0.0
    rng = np.random.default_rng(3)
    checked = 0
    for _ in range(400):
        i, j = rng.integers(0, m.n_panels, 2)
        if orc.classify(m.xyz, m.tri, int(i), int(j)) != 0:
            continue
        v = m.xyz[m.tri[j]]
        ref = high_order_dl_integral(v[0], v[1], v[2], nrm[j], c[i])
        got = orc.laplace_dl_entry(m.xyz, m.tri, int(i), int(j))
        assert abs(got - ref) <= 2e-3 * abs(ref) + 1e-9 * S[j], (i, j, got, ref)
        checked += 1
    assert checked > 200


@pytest.mark.parametrize("l,m", [(0, 0), (1, 1), (2, 0)])
def test_exterior_neumann_solve(orc, l, m):
    mesh = syn.sphere(3)
    Y = syn.ylm_rhs(mesh, l, m)
    g = -(l + 1) * Y                                   # du/dn of Y / r^(l+1) on r = 1
    b = -orc.matvec(orc.LAPLACE, mesh.xyz, mesh.tri, g)  # -V du/dn
    x, info, it, hist, tr = orc.solve(orc.LAPLACE_DL, mesh.xyz, mesh.tri, b, tol=1e-10)
    assert info == 0 and tr < 1e-9
    assert it <= 12                                    # second kind: few iterations
    err = np.linalg.norm(x - Y) / np.linalg.norm(Y)
    assert err < 2e-2, err
