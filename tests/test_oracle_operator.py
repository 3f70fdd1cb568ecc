"""Pins for the oracle's dense BEM operator and GMRES solve.

Closed forms (exact for the continuous sphere; the flat-panel discretisation
error must be small and must fall as the mesh is refined):
  * Laplace single layer with G = 1/(4 pi r) on the unit sphere:
    V[1] = 1 and V[Y_l^m] = Y_l^m / (2l+1) inside and on the sphere, so the
    density for phi = 1 is sigma = 1 and for phi = Y_l^m it is (2l+1) Y_l^m
    (Sec. 3.1 uses the phi = 1 case).
  * Stokes single layer (Eq. 6-7), int_S G_ij dS = (16 pi a / 3) delta_ij on a
    sphere of radius a, so a uniform traction t gives u = -(2a / 3 mu) t, the
    translating sphere has drag 6 pi mu a U (Sec. 3.2) and the rotating one
    torque -8 pi mu a^3 Omega.
Entry accuracy: every matrix entry against an independent high-order
integral of 1/r over its panel.
GMRES: against numpy's dense solver.
"""
import numpy as np
import pytest

import synthetic as syn


def high_order_panel_integral(v0, v1, v2, x, n=40):
    """int_T 1/|x - y| dA with an n x n collapsed Gauss-Legendre rule (x off the panel)."""
    g, w = np.polynomial.legendre.leggauss(n)
    s = 0.5 * (g + 1); ws = 0.5 * w
    S, Tt = np.meshgrid(s, s, indexing="ij")
    W = np.outer(ws, ws) * S
    l1 = S * (1 - Tt); l2 = S * Tt; l0 = 1 - S
    Y = l0[..., None] * v0 + l1[..., None] * v1 + l2[..., None] * v2
    area2 = np.linalg.norm(np.cross(v1 - v0, v2 - v0))
    return np.sum(W / np.linalg.norm(Y - x, axis=-1)) * area2


def test_laplace_constant_density(orc):
    errs = []
    for lev in (2, 3, 4):
        m = syn.sphere(lev)
        y = orc.matvec(orc.LAPLACE, m.xyz, m.tri, np.ones(m.n_panels))
        errs.append(np.max(np.abs(y - 1.0)))
    assert errs[-1] < 2e-3
    assert errs[0] > errs[1] > errs[2]


@pytest.mark.parametrize("l,m", [(1, 0), (2, 1), (3, -2), (4, 3)])
def test_laplace_ylm_eigenfunction(orc, l, m):
    errs = []
    for lev in (2, 3, 4):
        mesh = syn.sphere(lev)
        b = syn.ylm_rhs(mesh, l, m)
        y = orc.matvec(orc.LAPLACE, mesh.xyz, mesh.tri, b)
        c = syn.centroids(mesh)
        r = np.linalg.norm(c, axis=1)
        exact = r ** l * b / (2 * l + 1)
        errs.append(np.linalg.norm(y - exact) / np.linalg.norm(exact))
    # discretisation error, calibrated on this oracle: about 1.5e-3 (l+1) at 2048 panels
    assert errs[-1] < 2e-3 * (l + 1)
    assert errs[0] > errs[1] > errs[2]


def test_laplace_solve_sigma_one(orc):
    errs = []
    for lev in (2, 3, 4):
        m = syn.sphere(lev)
        x, info, it, hist, tr = orc.solve(orc.LAPLACE, m.xyz, m.tri, np.ones(m.n_panels), tol=1e-8)
        assert info == 0 and tr < 1e-7
        errs.append(np.linalg.norm(x - 1.0) / np.sqrt(m.n_panels))
    assert errs[0] > errs[1] > errs[2]
    assert errs[-1] < 2e-2


def test_laplace_solve_ylm(orc):
    mesh = syn.sphere(3)
    for l, m in syn.ylm_orders(0):
        b = syn.ylm_rhs(mesh, l, m)
        x, info, it, hist, tr = orc.solve(orc.LAPLACE, mesh.xyz, mesh.tri, b, tol=1e-8)
        assert info == 0
        err = np.linalg.norm(x - (2 * l + 1) * b) / np.linalg.norm((2 * l + 1) * b)
        assert err < 5e-2, (l, m, err)


def test_laplace_entries_against_independent_integral(orc):
    mesh = syn.sphere(3)
    c, S, _ = orc.panels(mesh.xyz, mesh.tri)
    b4, w4 = orc.far_rule()
    rng = np.random.default_rng(3)
    worst = {0: 0.0, 1: 0.0}
    worst_far_rule_on_near = 0.0
    count = {0: 0, 1: 0}
    for i in rng.choice(mesh.n_panels, 12, replace=False):
        row, cls = orc.laplace_row(mesh.xyz, mesh.tri, i)
        for j in range(mesh.n_panels):
            if i == j:
                assert cls[j] == 2
                continue
            d2 = np.sum((c[i] - c[j]) ** 2)
            assert cls[j] == (1 if d2 < 8 * S[j] else 0)
            v = mesh.xyz[mesh.tri[j]]
            ref = high_order_panel_integral(v[0], v[1], v[2], c[i])
            worst[cls[j]] = max(worst[cls[j]], abs(row[j] - ref) / ref)
            count[cls[j]] += 1
            if cls[j] == 1:
                y = b4 @ v
                four = np.sum(w4 * S[j] / np.linalg.norm(c[i] - y, axis=1))
                worst_far_rule_on_near = max(worst_far_rule_on_near, abs(four - ref) / ref)
    assert count[1] > 0 and count[0] > 0
    # calibrated: 25-point rule <= 2.6e-3 on edge neighbours, 4-point rule <= 1.3e-4 beyond
    # 2 sqrt(2 S_j); a wrong weight, point or index moves these by orders of magnitude
    assert worst[1] < 4e-3
    assert worst[0] < 3e-4
    assert worst_far_rule_on_near > 3 * worst[1]  # the near rule earns its place


def test_laplace_self_entry(orc):
    mesh = syn.sphere(2)
    c, S, _ = orc.panels(mesh.xyz, mesh.tri)
    for i in (0, 17, 100):
        v = mesh.xyz[mesh.tri[i]]
        assert orc.laplace_entry(mesh.xyz, mesh.tri, i, i) == orc.laplace_self(v[0], v[1], v[2], c[i])
        assert orc.classify(mesh.xyz, mesh.tri, i, i) == 2


def test_stokes_uniform_traction(orc):
    errs = []
    mu = 1.0
    for lev in (2, 3):
        m = syn.sphere(lev)
        t = np.tile([1.0, -0.5, 0.25], m.n_panels)
        u = orc.matvec(orc.STOKES, m.xyz, m.tri, t, mu=mu).reshape(-1, 3)
        exact = -(2.0 / (3.0 * mu)) * np.array([1.0, -0.5, 0.25])
        errs.append(np.max(np.abs(u - exact)) / np.linalg.norm(exact))
    assert errs[1] < errs[0] < 2e-2


def test_stokes_block_symmetry(orc):
    m = syn.sphere(2)
    # A_ij blocks are symmetric 3x3 matrices: probe with unit vectors on one panel
    rng = np.random.default_rng(1)
    j = 5
    cols = []
    for a in range(3):
        t = np.zeros(3 * m.n_panels)
        t[3 * j + a] = 1.0
        cols.append(orc.matvec(orc.STOKES, m.xyz, m.tri, t).reshape(-1, 3))
    blocks = np.stack(cols, axis=2)  # [i, p, a]
    assert np.max(np.abs(blocks - np.transpose(blocks, (0, 2, 1)))) < 1e-15


@pytest.mark.parametrize("mu", [1.0, 1e-3])
def test_stokes_drag_translating_sphere(orc, mu):
    errs = []
    for lev in (2, 3):
        m = syn.sphere(lev)
        u = np.tile([1.0, 0.0, 0.0], m.n_panels)
        t, info, it, hist, tr = orc.solve(orc.STOKES, m.xyz, m.tri, u, tol=1e-8, mu=mu)
        assert info == 0
        F, T = orc.force_torque(m.xyz, m.tri, t)
        exact = -6 * np.pi * mu
        errs.append(abs(F[0] - exact) / abs(exact))
        assert abs(F[1]) < 1e-6 * abs(exact) and abs(F[2]) < 1e-6 * abs(exact)
        # the refined octahedron is not mirror-symmetric, so a small torque remains
        assert np.max(np.abs(T)) < 1e-5 * abs(exact)
    # calibrated: 3.4e-2 at 128 panels, 8.9e-3 at 512
    assert errs[1] < errs[0] < 0.05
    assert errs[1] < 0.015


def test_stokes_torque_rotating_sphere(orc):
    m = syn.sphere(3)
    omega = np.array([0.0, 0.0, 1.0])
    c, S, _ = orc.panels(m.xyz, m.tri)
    u = np.cross(omega, c).reshape(-1)
    t, info, it, hist, tr = orc.solve(orc.STOKES, m.xyz, m.tri, u, tol=1e-8)
    assert info == 0
    F, T = orc.force_torque(m.xyz, m.tri, t)
    exact = -8 * np.pi
    # calibrated: 2.7e-2 at 512 panels (1.0e-1 at 128)
    assert abs(T[2] - exact) / abs(exact) < 0.04
    assert np.max(np.abs(F)) < 1e-5 * abs(exact)  # mesh chirality leaves a tiny net force


def test_gmres_matches_dense_solve(orc):
    rng = np.random.default_rng(11)
    n = 120
    A = np.eye(n) * 4 + rng.normal(size=(n, n)) / np.sqrt(n)
    b = rng.normal(size=n)
    x, info, it, hist, tr = orc.gmres(n, lambda v: A @ v, b, tol=1e-12, restart=50, max_iter=400)
    xr = np.linalg.solve(A, b)
    assert info == 0
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) < 1e-10
    assert np.all(np.diff(hist) <= 1e-15)  # GMRES residual never increases within a cycle


def test_gmres_exact_in_n_steps(orc):
    rng = np.random.default_rng(12)
    n = 30
    A = rng.normal(size=(n, n)) + 0.5 * np.eye(n)
    b = rng.normal(size=n)
    x, info, it, hist, tr = orc.gmres(n, lambda v: A @ v, b, tol=1e-13, restart=n, max_iter=n)
    assert info == 0 and it <= n
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) < 1e-10


def test_gmres_implicit_residual_is_true_residual(orc):
    rng = np.random.default_rng(13)
    n = 80
    A = np.eye(n) * 3 + rng.normal(size=(n, n)) / np.sqrt(n)
    b = rng.normal(size=n)
    # stop early by max_iter, compare the implicit estimate with |b - A x|
    x, info, it, hist, tr = orc.gmres(n, lambda v: A @ v, b, tol=1e-30, restart=80, max_iter=10)
    assert it == 10
    assert abs(hist[-1] - np.linalg.norm(b - A @ x) / np.linalg.norm(b)) < 1e-12
    assert abs(tr - hist[-1]) < 1e-12


def test_stokes_normal_field_is_near_null(orc):
    # incompressibility: a traction along the normal of a closed body induces no
    # velocity (int_S G n dS = 0), so the discrete operator nearly annihilates n
    m = syn.sphere(3)
    c, S, n = orc.panels(m.xyz, m.tri)
    un = orc.matvec(orc.STOKES, m.xyz, m.tri, n.reshape(-1))
    ue = orc.matvec(orc.STOKES, m.xyz, m.tri, np.tile([1.0, 0.0, 0.0], m.n_panels))
    assert np.linalg.norm(un) < 1e-4 * np.linalg.norm(ue)
