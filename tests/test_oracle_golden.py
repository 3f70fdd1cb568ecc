"""Oracle against values the paper prints (tests/golden/paper_values.json)."""
import json
import os

import numpy as np

import synthetic as syn

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_sphere_drag_printed_value(orc):
    g = GOLD["stokes_sphere_drag"]
    m = syn.sphere(4, radius=g["radius"])
    u = np.tile([g["U"], 0.0, 0.0], m.n_panels)
    t, info, it, hist, tr = orc.solve(orc.STOKES, m.xyz, m.tri, u, tol=1e-6, mu=g["mu"])
    assert info == 0
    F, _ = orc.force_torque(m.xyz, m.tri, t)
    # printed to 4 digits; 2048 panels carry ~2e-3 discretisation error
    assert abs(abs(F[0]) - g["F_d"]) / g["F_d"] < 5e-3
    assert abs(6 * np.pi * g["mu"] * g["radius"] * g["U"] - g["F_d"]) < 1e-5


def test_rbc_drag_printed_value(orc):
    g = GOLD["rbc_drag_512"]
    m = syn.rbc(3)
    assert m.n_panels == g["panels"]
    u = np.tile(g["U"], m.n_panels)
    t, info, it, hist, tr = orc.solve(orc.STOKES, m.xyz, m.tri, u, tol=1e-6, mu=g["mu"])
    assert info == 0
    F, _ = orc.force_torque(m.xyz, m.tri, t)
    # two printed digits: soft bound
    assert abs(F[0] - g["f_x"]) / abs(g["f_x"]) < 0.05


def test_laplace_sigma_printed(orc):
    m = syn.sphere(3)
    x, info, it, hist, tr = orc.solve(orc.LAPLACE, m.xyz, m.tri, np.ones(m.n_panels), tol=1e-8)
    assert np.max(np.abs(x - GOLD["laplace_sphere_density"]["sigma"])) < 0.05
