"""Python access to the oracle (plain FP64 CPU reference, see oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
bench's CPU-baseline leg; never by the product package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")
_SRC = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "tree.c")]

LAPLACE, STOKES, LAPLACE_DL = 0, 1, 2  # single layer, Stokes single layer, 1/2 I - K (exterior Neumann)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no FMA contraction)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    os.makedirs(_BUILD, exist_ok=True)
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", tmp] + _SRC + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        d, i32, i64, u64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        pd, pi32, pi64 = P(d), P(i32), P(i64)
        L.or_panels.argtypes = [i64, pd, pi32, pd, pd, pd]
        L.or_far_rule.argtypes = [pd, pd]
        L.or_near_rule.argtypes = [ctypes.c_int, pd, pd]
        L.or_gauss_legendre.argtypes = [ctypes.c_int, pd, pd]
        L.or_laplace_self.argtypes = [pd, pd, pd, pd]
        L.or_laplace_self.restype = d
        L.or_stokes_self.argtypes = [pd, pd, pd, pd, pd, pd]
        L.or_matvec_laplace.argtypes = [i64, pd, pi32, pd, pd, i64, pi64]
        L.or_matvec_stokes.argtypes = [i64, pd, pi32, d, pd, pd, i64, pi64]
        L.or_matvec_laplace_dl.argtypes = [i64, pd, pi32, pd, pd, i64, pi64]
        L.or_laplace_dl_entry.argtypes = [i64, pd, pi32, i64, i64]
        L.or_laplace_dl_entry.restype = d
        L.or_laplace_entry.argtypes = [i64, pd, pi32, i64, i64]
        L.or_laplace_entry.restype = d
        L.or_classify.argtypes = [i64, pd, pi32, i64, i64]
        L.or_laplace_row.argtypes = [i64, pd, pi32, i64, pd, pi32]
        L.or_gmres.argtypes = [i64, ctypes.c_void_p, ctypes.c_void_p, pd, d, ctypes.c_int,
                               ctypes.c_int, pd, pd, ctypes.c_int, P(ctypes.c_int), pd]
        L.or_solve.argtypes = [ctypes.c_int, i64, pd, pi32, d, pd, d, ctypes.c_int, ctypes.c_int,
                               pd, pd, ctypes.c_int, P(ctypes.c_int), pd]
        L.or_force_torque.argtypes = [i64, pd, pi32, pd, pd, pd]
        L.or_num_threads.restype = ctypes.c_int
        L.or_tree_build.argtypes = [i64, pd, pi32, i32, d]
        L.or_tree_build.restype = ctypes.c_void_p
        L.or_tree_sizes.argtypes = [ctypes.c_void_p, pi64]
        L.or_tree_get.argtypes = [ctypes.c_void_p, pi32, P(u64), pi32, pd, pi32, pi32, pd]
        L.or_tree_free.argtypes = [ctypes.c_void_p]
        _lib = L
    return _lib


def _p(a, ct=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _mesh_args(xyz, tri):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    return xyz, tri


def num_threads() -> int:
    return int(lib().or_num_threads())


def panels(xyz, tri):
    xyz, tri = _mesh_args(xyz, tri)
    nt = tri.shape[0]
    c = np.empty((nt, 3)); S = np.empty(nt); n = np.empty((nt, 3))
    lib().or_panels(nt, _p(xyz), _p(tri, ctypes.c_int32), _p(c), _p(S), _p(n))
    return c, S, n


def far_rule():
    b = np.empty((4, 3)); w = np.empty(4)
    lib().or_far_rule(_p(b), _p(w))
    return b, w


def near_rule(n1d: int = 5):
    b = np.empty((n1d * n1d, 3)); w = np.empty(n1d * n1d)
    k = lib().or_near_rule(n1d, _p(b), _p(w))
    assert k == n1d * n1d
    return b, w


def gauss_legendre(n: int):
    x = np.empty(n); w = np.empty(n)
    lib().or_gauss_legendre(n, _p(x), _p(w))
    return x, w


def laplace_self(v0, v1, v2, x) -> float:
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (v0, v1, v2, x)]
    return float(lib().or_laplace_self(*[_p(v) for v in a]))


def stokes_self(v0, v1, v2, x):
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (v0, v1, v2, x)]
    I = np.empty(1); J = np.empty(9)
    lib().or_stokes_self(*[_p(v) for v in a], _p(I), _p(J))
    return float(I[0]), J.reshape(3, 3)


def matvec(kernel: int, xyz, tri, x, mu: float = 1.0, rows=None):
    """Dense y = A x (rows=None) or the listed rows of it."""
    xyz, tri = _mesh_args(xyz, tri)
    nt = tri.shape[0]
    x = np.ascontiguousarray(x, dtype=np.float64)
    if rows is None:
        nr, rp = 0, None
        ny = nt
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        nr, rp = rows.shape[0], _p(rows, ctypes.c_int64)
        ny = nr
    if kernel == LAPLACE:
        y = np.empty(ny)
        rc = lib().or_matvec_laplace(nt, _p(xyz), _p(tri, ctypes.c_int32), _p(x), _p(y), nr, rp)
    elif kernel == LAPLACE_DL:
        y = np.empty(ny)
        rc = lib().or_matvec_laplace_dl(nt, _p(xyz), _p(tri, ctypes.c_int32), _p(x), _p(y), nr, rp)
    else:
        y = np.empty(3 * ny)
        rc = lib().or_matvec_stokes(nt, _p(xyz), _p(tri, ctypes.c_int32), mu, _p(x), _p(y), nr, rp)
    if rc != 0:
        raise MemoryError("oracle matvec failed")
    return y


def laplace_entry(xyz, tri, i: int, j: int) -> float:
    xyz, tri = _mesh_args(xyz, tri)
    return float(lib().or_laplace_entry(tri.shape[0], _p(xyz), _p(tri, ctypes.c_int32), i, j))


def laplace_dl_entry(xyz, tri, i: int, j: int) -> float:
    """int_j n_j . (x_i - y) / |x_i - y|^3 dA (no 1/(4 pi)) by the panel pair's rule."""
    xyz, tri = _mesh_args(xyz, tri)
    return float(lib().or_laplace_dl_entry(tri.shape[0], _p(xyz), _p(tri, ctypes.c_int32), i, j))


def laplace_row(xyz, tri, i: int):
    """Row i of int_j 1/r (no 1/(4 pi)) and the class of each entry."""
    xyz, tri = _mesh_args(xyz, tri)
    nt = tri.shape[0]
    out = np.empty(nt); cls = np.empty(nt, dtype=np.int32)
    lib().or_laplace_row(nt, _p(xyz), _p(tri, ctypes.c_int32), i, _p(out), _p(cls, ctypes.c_int32))
    return out, cls


def classify(xyz, tri, i: int, j: int) -> int:
    xyz, tri = _mesh_args(xyz, tri)
    return int(lib().or_classify(tri.shape[0], _p(xyz), _p(tri, ctypes.c_int32), i, j))


MV_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(ctypes.c_double))


def gmres(n: int, matvec_fn, b, tol: float, restart: int = 50, max_iter: int = 500):
    """GMRES(m) on a Python operator (tests); returns (x, info, iters, hist, true_res)."""
    b = np.ascontiguousarray(b, dtype=np.float64)

    def _cb(_u, xp, yp):
        xv = np.ctypeslib.as_array(xp, shape=(n,))
        yv = np.ctypeslib.as_array(yp, shape=(n,))
        yv[:] = matvec_fn(xv.copy())

    cb = MV_FN(_cb)
    x = np.empty(n); hist = np.zeros(max_iter); it = ctypes.c_int(0); tr = np.empty(1)
    info = lib().or_gmres(n, ctypes.cast(cb, ctypes.c_void_p), None, _p(b), tol, restart, max_iter,
                          _p(x), _p(hist), max_iter, ctypes.byref(it), _p(tr))
    return x, int(info), int(it.value), hist[: it.value].copy(), float(tr[0])


def solve(kernel: int, xyz, tri, b, tol: float = 1e-6, restart: int = 50, max_iter: int = 500,
          mu: float = 1.0):
    """Dense-operator GMRES solve; returns (x, info, iters, hist, true_res)."""
    xyz, tri = _mesh_args(xyz, tri)
    nt = tri.shape[0]
    n = 3 * nt if kernel == STOKES else nt
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty(n); hist = np.zeros(max_iter); it = ctypes.c_int(0); tr = np.empty(1)
    info = lib().or_solve(kernel, nt, _p(xyz), _p(tri, ctypes.c_int32), mu, _p(b), tol, restart,
                          max_iter, _p(x), _p(hist), max_iter, ctypes.byref(it), _p(tr))
    return x, int(info), int(it.value), hist[: it.value].copy(), float(tr[0])


def force_torque(xyz, tri, t):
    xyz, tri = _mesh_args(xyz, tri)
    t = np.ascontiguousarray(t, dtype=np.float64)
    F = np.empty(3); T = np.empty(3)
    lib().or_force_torque(tri.shape[0], _p(xyz), _p(tri, ctypes.c_int32), _p(t), _p(F), _p(T))
    return F, T


class Tree:
    """CPU reference octree and lists (see tree.c)."""

    def __init__(self, xyz, tri, ncrit: int, theta: float):
        xyz, tri = _mesh_args(xyz, tri)
        L = lib()
        h = L.or_tree_build(tri.shape[0], _p(xyz), _p(tri, ctypes.c_int32), ncrit, theta)
        if not h:
            raise ValueError("tree build failed")
        sz = np.empty(4, dtype=np.int64)
        L.or_tree_sizes(h, _p(sz, ctypes.c_int64))
        nbox, self.nlevels, nm, npp = (int(v) for v in sz)
        nt = tri.shape[0]
        self.perm = np.empty(nt, dtype=np.int32)
        self.keys = np.empty(nt, dtype=np.uint64)
        self.boxes = np.empty((nbox, 6), dtype=np.int32)
        self.box_real = np.empty((nbox, 5))
        self.m2l = np.empty((nm, 2), dtype=np.int32)
        self.p2p = np.empty((npp, 2), dtype=np.int32)
        self.cube = np.empty(4)
        L.or_tree_get(h, _p(self.perm, ctypes.c_int32), _p(self.keys, ctypes.c_uint64),
                      _p(self.boxes, ctypes.c_int32), _p(self.box_real),
                      _p(self.m2l, ctypes.c_int32), _p(self.p2p, ctypes.c_int32), _p(self.cube))
        L.or_tree_free(h)

    @property
    def nbox(self) -> int:
        return self.boxes.shape[0]
