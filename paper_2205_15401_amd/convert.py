"""Mesh and point-cloud converters: Gaussian ellipsoids from triangle meshes
and point sets (Sec. 3.2, "VoGE mesh converter"; App. "Mesh & Point Cloud
Converter").  Host-side numpy; the outputs are the float32 (means, packed
covariances) the renderer takes.

Mesh: one kernel per vertex, centred on it.  With d_k the mean length of
the edges at vertex k and the coverage rate zeta, the isotropic covariance is
Sigma_k = sigma_k I with sigma_k = (d_k / 2)^2 / ln(1/zeta) (the appendix's
equation; Sec. 3.2 writes the same value as l^2 / (4 ln(1/zeta))).  The
optional flattening turns the sphere into an ellipsoid flat along the
surface: the variance along the vertex normal n is multiplied by the flatten
rate f, Sigma_k = sigma_k (I - (1 - f) n n^T), i.e. R diag(s, s, f s) R^T
for any rotation R whose third column is n.

Point cloud: the same sigma_k with d_k the mean distance from point k to its
m nearest other points.
"""

from __future__ import annotations

import math
from typing import Optional, Tuple

import numpy as np


def _packed(full: np.ndarray) -> np.ndarray:
    return np.stack([full[:, 0, 0], full[:, 0, 1], full[:, 0, 2], full[:, 1, 1], full[:, 1, 2], full[:, 2, 2]],
                    axis=1)


def sigma_from_spacing(d: np.ndarray, zeta: float) -> np.ndarray:
    """sigma = (d/2)^2 / ln(1/zeta), the per-axis variance of a converted kernel."""
    if not 0.0 < zeta < 1.0:
        raise ValueError("zeta must be in (0, 1)")
    d = np.asarray(d, np.float64)
    return (0.5 * d) ** 2 / math.log(1.0 / zeta)


def mesh_edges(faces: np.ndarray) -> np.ndarray:
    """Undirected edges (E, 2), each once, of a triangle list (F, 3)."""
    f = np.asarray(faces, np.int64)
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
    e = np.sort(e, axis=1)
    return np.unique(e, axis=0)


def vertex_normals(verts: np.ndarray, faces: np.ndarray) -> np.ndarray:
    """Unit vertex normals: sums of the adjacent faces' area-weighted normals."""
    v = np.asarray(verts, np.float64)
    f = np.asarray(faces, np.int64)
    fn = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])    # length = 2 x area
    n = np.zeros_like(v)
    for c in range(3):
        np.add.at(n, f[:, c], fn)
    ln = np.linalg.norm(n, axis=1, keepdims=True)
    return n / np.where(ln > 0, ln, 1.0)


def mesh_to_gaussians(verts: np.ndarray, faces: np.ndarray, zeta: float = 0.5,
                      flatten: Optional[float] = None) -> Tuple[np.ndarray, np.ndarray]:
    """Kernels at the mesh vertices.  Returns (means (V, 3), packed covs (V, 6)),
    float32.  flatten: None for spheres, else the rate in (0, 1] applied to the
    variance along the vertex normal."""
    v = np.asarray(verts, np.float64)
    e = mesh_edges(faces)
    length = np.linalg.norm(v[e[:, 0]] - v[e[:, 1]], axis=1)
    total = np.zeros(v.shape[0])
    count = np.zeros(v.shape[0])
    for c in range(2):
        np.add.at(total, e[:, c], length)
        np.add.at(count, e[:, c], 1.0)
    if np.any(count == 0):
        raise ValueError("every vertex needs at least one edge")
    sig = sigma_from_spacing(total / count, zeta)
    full = sig[:, None, None] * np.eye(3)[None]
    if flatten is not None:
        if not 0.0 < flatten <= 1.0:
            raise ValueError("flatten must be in (0, 1]")
        n = vertex_normals(v, faces)
        full = full - (1.0 - flatten) * sig[:, None, None] * np.einsum("ni,nj->nij", n, n)
    return v.astype(np.float32), _packed(full).astype(np.float32)


def pointcloud_to_gaussians(points: np.ndarray, m: int = 3, zeta: float = 0.5) -> Tuple[np.ndarray, np.ndarray]:
    """Isotropic kernels at the points; d_k = mean distance to the m nearest
    other points."""
    from scipy.spatial import cKDTree

    p = np.asarray(points, np.float64)
    if p.shape[0] < m + 1:
        raise ValueError("need more than m points")
    dist, _ = cKDTree(p).query(p, k=m + 1)          # the first neighbour is the point itself
    sig = sigma_from_spacing(dist[:, 1:].mean(axis=1), zeta)
    full = sig[:, None, None] * np.eye(3)[None]
    return p.astype(np.float32), _packed(full).astype(np.float32)


def icosphere(subdivisions: int = 4, radius: float = 1.0) -> Tuple[np.ndarray, np.ndarray]:
    """Sphere mesh by repeated 4-to-1 splits of an icosahedron, vertices pushed
    to the sphere: 10 * 4^s + 2 vertices (2,562 at s = 4).  Returns
    (verts (V, 3) float64, faces (F, 3) int64), faces counter-clockwise seen
    from outside."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
             (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5), (2, 4, 11),
             (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    v = [np.asarray(p, np.float64) / np.linalg.norm(p) for p in verts]
    f = list(faces)
    for _ in range(subdivisions):
        mid = {}

        def midpoint(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in mid:
                p = v[a] + v[b]
                v.append(p / np.linalg.norm(p))
                mid[key] = len(v) - 1
            return mid[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = nf
    return radius * np.stack(v), np.asarray(f, np.int64)
