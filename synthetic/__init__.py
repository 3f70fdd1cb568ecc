"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the method itself (no quadrature, no kernel
evaluation, no tree): it only produces the inputs the paper's experiments are
run on, namely triangulated surfaces, boundary data at the collocation points
and random vectors.

* Sphere: an 8-triangle octahedron whose triangles are split into four,
  recursively, with new vertices pushed onto the sphere after each split
  (Sec. 3.1, grid-convergence study).  N = 8 * 4**k panels.
* Ellipsoid: the sphere mesh with vertices scaled per axis.
* Red blood cell: the sphere mesh mapped by the Evans-Fung biconcave profile,
  Eq. (21) (Sec. 3.3), r = 3.91, C0 = 0.81, C2 = 7.83, C4 = -4.39 (micrometres).
* Multi-cell scene: copies of one cell, each randomly rotated and shifted by a
  positive amount so that no two overlap (Sec. 3.3).

Triangles are listed counter-clockwise seen from outside the body, so the
right-hand-rule normal points out.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Mesh", "sphere", "ellipsoid", "rbc", "rbc_scene", "merge",
    "centroids", "real_ylm", "ylm_rhs", "ylm_orders", "random_vector",
    "RBC_R", "RBC_C0", "RBC_C2", "RBC_C4", "Request", "request_stream",
]


@dataclass
class Mesh:
    xyz: np.ndarray  # [nv, 3] float64
    tri: np.ndarray  # [nt, 3] int32, CCW seen from outside

    @property
    def n_panels(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n_vertices(self) -> int:
        return int(self.xyz.shape[0])


def _octahedron():
    v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                 dtype=np.float64)
    # counter-clockwise seen from outside: (a, b, c) with (b-a) x (c-a) pointing out
    px, nx, py, ny, pz, nz = range(6)
    t = [(px, py, pz), (py, nx, pz), (nx, ny, pz), (ny, px, pz),
         (py, px, nz), (nx, py, nz), (ny, nx, nz), (px, ny, nz)]
    return v, np.array(t, dtype=np.int64)


def sphere(level: int, radius: float = 1.0) -> Mesh:
    """Octahedron refined `level` times: 8 * 4**level panels on a sphere."""
    if level < 0:
        raise ValueError("level must be >= 0")
    v, t = _octahedron()
    verts = [tuple(p) for p in v]
    for _ in range(level):
        edge_mid = {}
        new_t = []

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = edge_mid.get(key)
            if idx is None:
                p = (np.array(verts[a]) + np.array(verts[b])) * 0.5
                p = p / np.linalg.norm(p)
                verts.append(tuple(p))
                idx = len(verts) - 1
                edge_mid[key] = idx
            return idx

        for a, b, c in t:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_t += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        t = np.array(new_t, dtype=np.int64)
    xyz = np.array(verts, dtype=np.float64) * float(radius)
    return Mesh(xyz=np.ascontiguousarray(xyz), tri=np.ascontiguousarray(t.astype(np.int32)))


def sphere_level_for(n_panels: int) -> int:
    k = 0
    while 8 * 4 ** k < n_panels:
        k += 1
    if 8 * 4 ** k != n_panels:
        raise ValueError(f"{n_panels} is not 8*4**k")
    return k


def ellipsoid(level: int, axes=(1.0, 1.0, 1.0)) -> Mesh:
    m = sphere(level)
    xyz = m.xyz * np.asarray(axes, dtype=np.float64)[None, :]
    return Mesh(xyz=np.ascontiguousarray(xyz), tri=m.tri)


RBC_R, RBC_C0, RBC_C2, RBC_C4 = 3.91, 0.81, 7.83, -4.39


def rbc(level: int) -> Mesh:
    """Evans-Fung biconcave cell, Eq. (21), from the unit-sphere mesh.

    x' = r x, y' = r y, rho = |(x', y')|, z' = +-1/2 sqrt(1-(rho/r)^2) (C0 + C2 (rho/r)^2
    + C4 (rho/r)^4), with the sign of the sphere vertex' z.  Where rounding makes
    1 - (rho/r)^2 negative it is taken as 0.
    """
    m = sphere(level)
    x, y, z = m.xyz[:, 0], m.xyz[:, 1], m.xyz[:, 2]
    s2 = x * x + y * y  # (rho / r)^2
    root = np.sqrt(np.maximum(0.0, 1.0 - s2))
    zz = np.sign(z) * 0.5 * root * (RBC_C0 + RBC_C2 * s2 + RBC_C4 * s2 * s2)
    xyz = np.stack([x * RBC_R, y * RBC_R, zz], axis=1)
    return Mesh(xyz=np.ascontiguousarray(xyz), tri=m.tri)


def merge(meshes) -> Mesh:
    xyz, tri, off = [], [], 0
    for m in meshes:
        xyz.append(m.xyz)
        tri.append(m.tri.astype(np.int64) + off)
        off += m.xyz.shape[0]
    return Mesh(xyz=np.ascontiguousarray(np.concatenate(xyz)),
                tri=np.ascontiguousarray(np.concatenate(tri).astype(np.int32)))


def _quat_to_rot(q):
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def rbc_scene(n_cells: int, level: int, seed: int, box: float = 60.0,
              margin: float = 4.5, gap: float = 0.5) -> Mesh:
    """`n_cells` copies of one cell, uniformly random orientation (normalised
    Gaussian quaternion) and centres uniform in [margin, box - margin]^3.  A
    centre closer than 2 (r + gap) to an earlier one is drawn again, so the cells'
    bounding spheres keep a gap and never overlap."""
    rng = np.random.default_rng(seed)
    cell = rbc(level)
    min_d = 2.0 * (RBC_R + gap)
    centres, meshes = [], []
    for _ in range(n_cells):
        q = rng.normal(size=4)
        q = q / np.linalg.norm(q)
        rot = _quat_to_rot(q)
        for _attempt in range(100000):
            c = rng.uniform(margin, box - margin, size=3)
            if all(np.linalg.norm(c - o) >= min_d for o in centres):
                break
        else:  # pragma: no cover - packing here is ~9% by volume
            raise RuntimeError("could not place cells without overlap")
        centres.append(c)
        meshes.append(Mesh(xyz=cell.xyz @ rot.T + c[None, :], tri=cell.tri))
    return merge(meshes)


def centroids(mesh: Mesh) -> np.ndarray:
    """Collocation points, used here only to evaluate boundary data."""
    v = mesh.xyz[mesh.tri]
    return (v[:, 0] + v[:, 1] + v[:, 2]) / 3.0


def real_ylm(l: int, m: int, pts: np.ndarray) -> np.ndarray:
    """Real orthonormal spherical harmonic Y_l^m at the directions of `pts`."""
    from scipy.special import sph_harm_y
    p = np.asarray(pts, dtype=np.float64)
    r = np.linalg.norm(p, axis=1)
    theta = np.arccos(np.clip(p[:, 2] / r, -1.0, 1.0))
    phi = np.arctan2(p[:, 1], p[:, 0])
    y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2.0) * (-1) ** m * y.real
    if m < 0:
        return math.sqrt(2.0) * (-1) ** m * y.imag
    return y.real


def ylm_orders(seed: int, lmax: int = 4):
    """(l, m_l) for l = 0..lmax with m_l drawn from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return [(l, int(rng.integers(-l, l + 1))) for l in range(lmax + 1)]


def ylm_rhs(mesh: Mesh, l: int, m: int) -> np.ndarray:
    return np.ascontiguousarray(real_ylm(l, m, centroids(mesh)))


def random_vector(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(n)


@dataclass
class Request:
    ticket: int
    arrival_s: float
    kernel: str      # "laplace" | "stokes"
    shape: str       # "sphere" | "ellipsoid" | "rbc"
    level: int       # panels = 8 * 4**level
    axes: tuple

    def mesh(self) -> Mesh:
        if self.shape == "sphere":
            return sphere(self.level)
        if self.shape == "ellipsoid":
            return ellipsoid(self.level, self.axes)
        return rbc(self.level)


def request_stream(n: int, rate_hz: float, seed: int, levels=(3, 4, 5, 6)):
    """Poisson arrivals of solve requests: kernel Laplace/Stokes with
    probability 1/2 each, shape sphere/ellipsoid/RBC with 1/3 each, ellipsoid
    axes uniform in [0.5, 2], panel counts 8 * 4**k with k uniform in `levels`."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        kernel = "laplace" if rng.random() < 0.5 else "stokes"
        shape = ("sphere", "ellipsoid", "rbc")[int(rng.integers(0, 3))]
        level = int(rng.choice(np.asarray(levels)))
        axes = tuple(float(a) for a in rng.uniform(0.5, 2.0, size=3))
        out.append(Request(i, t, kernel, shape, level, axes))
    return out
