"""Helpers for the GPU tests (device vectors, oracle references, meshes)."""
import numpy as np
import torch

import synthetic as syn


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev())


def rel_l2(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b):
    """largest element-wise difference over the largest reference element: a
    wrong leaf or panel, which a norm over many can hide, shows here"""
    a = np.asarray(a); b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def announce(msg):
    print(msg, flush=True)


MESHES = {
    "sphere512": lambda: syn.sphere(3),
    "sphere2048": lambda: syn.sphere(4),
    "sphere8192": lambda: syn.sphere(5),
    "rbc2048": lambda: syn.rbc(4),
    "ellipsoid2048": lambda: syn.ellipsoid(4, (0.6, 1.3, 1.9)),
    "cells8x512": lambda: syn.rbc_scene(8, 3, 1),
}


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


def compare(orc, kernel, mesh_name, m, x, xo, elementwise=False):
    """relative L2 error of x against the oracle solution, null-space free for
    Stokes (with elementwise: also the largest element's error, max_rel).

    The first-kind Stokes single layer maps the normal field of each closed
    body to (nearly) zero, so a traction is fixed only up to one multiple of
    the normal per body, which GMRES picks along its own Krylov path: Stokes
    solutions are compared after removing, body by body, their area-weighted
    normal component, and through the force on each body (which the normal
    field does not change)."""
    if kernel != 1:
        e = rel_l2(x, xo)
        return (e, max_rel(x, xo)) if elementwise else e
    bodies = bodies_of(mesh_name, m.n_panels)
    a, b = strip_normal(orc, m, x, bodies), strip_normal(orc, m, xo, bodies)
    e = rel_l2(a, b)
    Fo = body_forces(orc, m, xo, bodies)
    eF = float(np.max(np.abs(body_forces(orc, m, x, bodies) - Fo)) / np.max(np.abs(Fo)))
    return (max(e, eF), max_rel(a, b)) if elementwise else max(e, eF)
