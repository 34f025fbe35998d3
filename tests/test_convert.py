"""Mesh and point-cloud converters (Sec. 3.2; App. "Mesh & Point Cloud
Converter") against closed forms on regular meshes and lattices."""

import math

import numpy as np
import pytest

from paper_2205_15401_amd import convert as CV
from paper_2205_15401_amd import scenes as S


def grid_mesh(n, h):
    """n x n vertices in the plane z = 0, spacing h, each square split along
    the same diagonal."""
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    verts = np.stack([ii.ravel() * h, jj.ravel() * h, np.zeros(n * n)], axis=1)
    idx = lambda i, j: i * n + j  # noqa: E731
    faces = []
    for i in range(n - 1):
        for j in range(n - 1):
            faces += [(idx(i, j), idx(i + 1, j), idx(i + 1, j + 1)), (idx(i, j), idx(i + 1, j + 1), idx(i, j + 1))]
    return verts, np.asarray(faces)


@pytest.mark.parametrize("s, nv", [(0, 12), (1, 42), (2, 162), (3, 642), (4, 2562)])
def test_icosphere_counts_and_shape(s, nv):
    v, f = CV.icosphere(s, radius=2.0)
    assert v.shape == (nv, 3) and f.shape == (20 * 4 ** s, 3)
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), 2.0, rtol=1e-12)
    e = CV.mesh_edges(f)
    assert nv - e.shape[0] + f.shape[0] == 2                     # Euler characteristic of a sphere
    n = CV.vertex_normals(v, f)
    assert np.all(np.einsum("ij,ij->i", n, v / 2.0) > 0.99)      # outward, nearly radial


def test_mesh_sigma_on_a_regular_grid():
    """An interior vertex of the grid has four edges of length h and two
    diagonals h sqrt 2: d = (4 + 2 sqrt 2) h / 6, sigma = (d/2)^2 / ln(1/zeta)."""
    h, zeta = 0.1, 0.5
    verts, faces = grid_mesh(6, h)
    means, covs = CV.mesh_to_gaussians(verts, faces, zeta)
    d = (4 + 2 * math.sqrt(2)) * h / 6
    sig = (d / 2) ** 2 / math.log(1 / zeta)
    k = 2 * 6 + 3                                                 # an interior vertex
    np.testing.assert_allclose(covs[k], [sig, 0, 0, sig, 0, sig], rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(means, verts, rtol=0, atol=1e-7)
    # the coverage reading: at distance d/2 the density is sqrt(zeta) of the peak
    assert abs(math.exp(-(d / 2) ** 2 / (2 * sig)) - math.sqrt(zeta)) < 1e-12


def test_flattened_kernels_are_flat_along_the_normal():
    f = 0.1
    verts, faces = grid_mesh(5, 0.2)
    _, covs = CV.mesh_to_gaussians(verts, faces, 0.5, flatten=f)
    _, iso = CV.mesh_to_gaussians(verts, faces, 0.5)
    full = S.unpack_cov(covs)
    s = iso[:, 0]
    np.testing.assert_allclose(full[:, 2, 2], f * s, rtol=1e-6)   # the grid's normal is z
    np.testing.assert_allclose(full[:, 0, 0], s, rtol=1e-6)
    v, fc = CV.icosphere(2)
    _, cs = CV.mesh_to_gaussians(v, fc, 0.5, flatten=f)
    w, q = np.linalg.eigh(S.unpack_cov(cs).astype(np.float64))
    radial = v / np.linalg.norm(v, axis=1, keepdims=True)
    assert np.all(np.abs(np.einsum("ij,ij->i", q[:, :, 0], radial)) > 0.99)   # smallest axis ~ radial
    np.testing.assert_allclose(w[:, 0] / w[:, 2], f, rtol=1e-4)
    np.testing.assert_allclose(w[:, 1], w[:, 2], rtol=1e-4)


def test_pointcloud_sigma_on_a_lattice():
    """Every point of a cubic lattice has at least three neighbours at the
    spacing h, so with m = 3 each d_k is h."""
    h = 0.05
    g = np.arange(4) * h
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    _, covs = CV.pointcloud_to_gaussians(pts, m=3, zeta=0.3)
    sig = (h / 2) ** 2 / math.log(1 / 0.3)
    np.testing.assert_allclose(covs[:, [0, 3, 5]], sig, rtol=1e-5)
    assert np.all(covs[:, [1, 2, 4]] == 0)


def test_converter_arguments():
    verts, faces = grid_mesh(3, 1.0)
    with pytest.raises(ValueError):
        CV.mesh_to_gaussians(verts, faces, zeta=1.0)
    with pytest.raises(ValueError):
        CV.mesh_to_gaussians(verts, faces, flatten=0.0)
    with pytest.raises(ValueError):
        CV.pointcloud_to_gaussians(np.zeros((2, 3)), m=3)
