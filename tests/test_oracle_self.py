"""Pins for the oracle's integrals over the panel holding the target (Sec. 2.3).

* Equilateral triangle, target at the centroid: int 1/r dA = sqrt(3) s ln(2 + sqrt 3)
  (closed form), and J = int e e^T / r dA = (I/2) times the in-plane projector
  (three-fold symmetry plus trace J = I).
* Random triangles: against a brute-force Duffy integral.  Splitting the
  triangle at the target and collapsing each piece onto it cancels the 1/r
  singularity, leaving a smooth 1-D integral that scipy's adaptive quadrature
  evaluates to ~1e-14.
"""
import numpy as np
from scipy.integrate import quad


def duffy_reference(v0, v1, v2, x):
    I = 0.0
    J = np.zeros((3, 3))
    V = [v0, v1, v2]
    for e in range(3):
        a, b = V[e], V[(e + 1) % 3]
        jac = np.linalg.norm(np.cross(a - x, b - a))

        def d(t):
            return (a - x) + t * (b - a)

        I += quad(lambda t: jac / np.linalg.norm(d(t)), 0, 1, epsabs=1e-15, epsrel=1e-14, limit=200)[0]
        for p in range(3):
            for q in range(3):
                J[p, q] += quad(lambda t: jac * d(t)[p] * d(t)[q] / np.linalg.norm(d(t)) ** 3, 0, 1,
                                epsabs=1e-15, epsrel=1e-14, limit=200)[0]
    return I, J


def test_equilateral_closed_form(orc):
    for s in (1.0, 0.37, 5.0):
        v0 = np.array([0.0, 0.0, 0.0])
        v1 = np.array([s, 0.0, 0.0])
        v2 = np.array([s / 2, np.sqrt(3) / 2 * s, 0.0])
        c = (v0 + v1 + v2) / 3
        I = orc.laplace_self(v0, v1, v2, c)
        exact = np.sqrt(3) * s * np.log(2 + np.sqrt(3))
        assert abs(I - exact) < 1e-13 * exact
        I2, J = orc.stokes_self(v0, v1, v2, c)
        assert abs(I2 - I) < 1e-15 * exact
        P = np.diag([1.0, 1.0, 0.0])
        assert np.max(np.abs(J - 0.5 * I * P)) < 1e-13 * exact


def test_random_triangles_vs_duffy(orc):
    rng = np.random.default_rng(7)
    worst_I, worst_J = 0.0, 0.0
    for _ in range(100):
        v = rng.normal(size=(3, 3))
        # keep triangles away from degenerate slivers
        n = np.cross(v[1] - v[0], v[2] - v[0])
        if np.linalg.norm(n) < 0.2:
            continue
        c = v.mean(axis=0)
        I, J = orc.stokes_self(v[0], v[1], v[2], c)
        Ir, Jr = duffy_reference(v[0], v[1], v[2], c)
        worst_I = max(worst_I, abs(I - Ir) / Ir)
        worst_J = max(worst_J, np.max(np.abs(J - Jr)) / Ir)
        # invariants: trace J = I, J n = 0 (e lies in the panel's plane)
        nh = n / np.linalg.norm(n)
        assert abs(np.trace(J) - I) < 1e-13 * I
        assert np.max(np.abs(J @ nh)) < 1e-13 * I
        assert abs(orc.laplace_self(v[0], v[1], v[2], c) - I) < 1e-15 * I
    assert worst_I < 1e-12
    assert worst_J < 1e-12


def test_self_integral_scales_linearly(orc):
    v = np.array([[0.1, 0.2, 0.3], [1.3, -0.2, 0.5], [0.4, 1.1, -0.3]])
    c = v.mean(axis=0)
    I1 = orc.laplace_self(v[0], v[1], v[2], c)
    I2 = orc.laplace_self(3 * v[0], 3 * v[1], 3 * v[2], 3 * c)
    assert abs(I2 - 3 * I1) < 1e-13 * I2
