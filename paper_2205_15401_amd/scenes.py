"""Seeded synthetic inputs for the VoGE rendering path.

This module builds scenes (Gaussian-ellipsoid centres, covariances and
per-kernel attributes), pinhole cameras and upstream image gradients.  It is
the only code shared by the FP64 oracle and the GPU path, so it holds none of
the renderer's arithmetic: no ray tracing, no quadratic forms, no
transmittance.  Everything is numpy, float32 on output, and driven by
``numpy.random.default_rng(seed)``.

Conventions (the paper's notation, Sec. 3.3):
  * A kernel k has centre M_k (3 floats) and covariance Sigma_k, passed packed
    as 6 floats (xx, xy, xz, yy, yz, zz).
  * The camera maps world to camera space as X_cam = R X + T (Eq. 3) and has
    focal length F and principal point (O_x, O_y) in pixels.  The ray of pixel
    (i, j) -- i the row, j the column -- has direction
    ((i - O_y)/F, (j - O_x)/F, 1) (Eq. 5); camera x runs down the rows,
    camera y along the columns, z is the viewing direction.
  * Sizes called "sigma" or "axis" below are standard deviations:
    Sigma = Q diag(s^2) Q^T.

Workloads (their shapes follow the paper's speed study, Fig. fig:speed, and
its converted CAD objects and point clouds, Sec. 4 and App. B):
  * ``config_small``   64x64, 512 isotropic kernels, K=16, forward only.
  * ``config_torus``   512x512, 10,000 thin anisotropic kernels on a torus,
                       16 channels, K=20, forward + backward.
  * ``config_poses``   one 4,096-kernel torus seen from 256 look-at poses at
                       128x128, K=20.
  * ``config_uneven``  64 random ellipsoid clouds of 1k-100k kernels, image
                       sizes 64..512, K in {8, 16, 32}.
  * ``config_serving`` resident scenes of 10k..200k kernels and a request mix.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

ETA_DEFAULT = 0.01  # density threshold eta of the fine stage (App. A.3)
K_DEFAULT = 20      # K' nearest kernels kept per ray (App. A.3)


@dataclasses.dataclass
class Camera:
    """Pinhole camera: extrinsics (R, T) and intrinsics (F, O_x, O_y)."""

    R: np.ndarray          # (3, 3) float32, world -> camera rotation
    T: np.ndarray          # (3,) float32, translation
    focal: float           # F in pixels
    cx: float              # O_x, principal point column
    cy: float              # O_y, principal point row
    height: int
    width: int

    def as_vector(self) -> np.ndarray:
        """(R row-major 9, T 3, F, O_x, O_y) as float32, the packed camera order."""
        return np.concatenate([
            np.asarray(self.R, np.float32).reshape(9),
            np.asarray(self.T, np.float32).reshape(3),
            np.array([self.focal, self.cx, self.cy], np.float32),
        ]).astype(np.float32)

    @staticmethod
    def from_vector(vec, height: int, width: int) -> "Camera":
        v = np.asarray(vec, np.float32).reshape(15)
        return Camera(R=v[:9].reshape(3, 3).copy(), T=v[9:12].copy(),
                      focal=float(v[12]), cx=float(v[13]), cy=float(v[14]),
                      height=int(height), width=int(width))


@dataclasses.dataclass
class Scene:
    """A set of Gaussian ellipsoids (the kernel set of Sec. 3.2)."""

    means: np.ndarray      # (N, 3) float32
    covs: np.ndarray       # (N, 6) float32 packed xx, xy, xz, yy, yz, zz
    attrs: np.ndarray      # (N, C) float32

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def channels(self) -> int:
        return int(self.attrs.shape[1])


@dataclasses.dataclass
class Job:
    """One render request: a scene, a camera, K, eta and an optional upstream gradient."""

    scene: Scene
    camera: Camera
    K: int = K_DEFAULT
    eta: float = ETA_DEFAULT
    grad_image: Optional[np.ndarray] = None   # (H, W, C) float32
    name: str = ""


# --------------------------------------------------------------------------
# small building blocks
# --------------------------------------------------------------------------

def pack_cov(full: np.ndarray) -> np.ndarray:
    """(N,3,3) symmetric -> (N,6) packed xx, xy, xz, yy, yz, zz."""
    f = np.asarray(full)
    return np.stack([f[:, 0, 0], f[:, 0, 1], f[:, 0, 2],
                     f[:, 1, 1], f[:, 1, 2], f[:, 2, 2]], axis=1)


def unpack_cov(packed: np.ndarray) -> np.ndarray:
    """(N,6) packed -> (N,3,3) symmetric."""
    p = np.asarray(packed)
    xx, xy, xz, yy, yz, zz = (p[:, i] for i in range(6))
    return np.stack([np.stack([xx, xy, xz], -1),
                     np.stack([xy, yy, yz], -1),
                     np.stack([xz, yz, zz], -1)], axis=1)


def covariance_from_axes(frames: np.ndarray, stds: np.ndarray) -> np.ndarray:
    """Sigma = Q diag(std^2) Q^T for per-kernel orthonormal frames Q (columns = axes)."""
    Q = np.asarray(frames, np.float64)
    s2 = np.asarray(stds, np.float64) ** 2
    full = np.einsum("nij,nj,nkj->nik", Q, s2, Q)
    return pack_cov(full).astype(np.float32)


def random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform rotations on SO(3) from normalised Gaussian quaternions."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], axis=1)


def identity_camera(size: int, focal: Optional[float] = None, height: Optional[int] = None) -> Camera:
    """Camera at the origin looking down +z, principal point at the image centre."""
    h = int(height if height is not None else size)
    w = int(size)
    f = float(focal if focal is not None else w)
    return Camera(R=np.eye(3, dtype=np.float32), T=np.zeros(3, np.float32),
                  focal=f, cx=w / 2.0, cy=h / 2.0, height=h, width=w)


def look_at_camera(position: np.ndarray, size: int, focal: Optional[float] = None,
                   target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)) -> Camera:
    """Camera at ``position`` looking at ``target``.

    Rows of R are the camera axes in world coordinates: z = viewing direction,
    x = image-down (rows), y = z cross x so that R is a proper rotation.
    T = -R position.
    """
    pos = np.asarray(position, np.float64)
    fwd = np.asarray(target, np.float64) - pos
    fwd /= np.linalg.norm(fwd)
    upv = np.asarray(up, np.float64)
    upv = upv - fwd * np.dot(upv, fwd)
    upv /= np.linalg.norm(upv)
    x_ax = -upv
    y_ax = np.cross(fwd, x_ax)
    R = np.stack([x_ax, y_ax, fwd], axis=0)
    T = -R @ pos
    w = int(size)
    f = float(focal if focal is not None else w)
    return Camera(R=R.astype(np.float32), T=T.astype(np.float32), focal=f,
                  cx=w / 2.0, cy=w / 2.0, height=w, width=w)


# --------------------------------------------------------------------------
# scene generators
# --------------------------------------------------------------------------

TORUS_AXIS = np.array([0.0, 1.0, -1.0]) / math.sqrt(2.0)


def torus_scene(rng: np.random.Generator, n: int, channels: int, centre=(0.0, 0.0, 3.0),
                major: float = 1.0, minor: float = 0.35,
                axis_stds=(0.03, 0.03, 0.006), attr_dist: str = "normal") -> Scene:
    """Kernels area-uniform on a torus surface, flattened along the surface normal.

    Each kernel's frame is (t1, t2, n) with n the surface normal and (t1, t2)
    the tangent plane turned by a random angle; its standard deviations along
    those axes are ``axis_stds`` (the flattened ellipsoids of the mesh
    converter, Sec. 3.2 and App. A.4).
    """
    ax = TORUS_AXIS
    # an orthonormal pair spanning the torus plane
    e1 = np.cross(ax, [1.0, 0.0, 0.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(ax, e1)
    u = rng.uniform(0.0, 2.0 * math.pi, n)
    # v with density proportional to (R + r cos v): rejection sampling
    v = np.empty(n)
    filled = 0
    while filled < n:
        cand = rng.uniform(0.0, 2.0 * math.pi, 2 * (n - filled) + 16)
        acc = rng.uniform(0.0, major + minor, cand.shape[0]) < (major + minor * np.cos(cand))
        take = cand[acc][: n - filled]
        v[filled:filled + take.shape[0]] = take
        filled += take.shape[0]
    radial = np.cos(u)[:, None] * e1 + np.sin(u)[:, None] * e2
    pos = np.asarray(centre, np.float64) + (major + minor * np.cos(v))[:, None] * radial \
        + (minor * np.sin(v))[:, None] * ax
    normal = np.cos(v)[:, None] * radial + np.sin(v)[:, None] * ax
    t_u = -np.sin(u)[:, None] * e1 + np.cos(u)[:, None] * e2
    t_v = np.cross(normal, t_u)
    theta = rng.uniform(0.0, 2.0 * math.pi, n)
    t1 = np.cos(theta)[:, None] * t_u + np.sin(theta)[:, None] * t_v
    t2 = -np.sin(theta)[:, None] * t_u + np.cos(theta)[:, None] * t_v
    frames = np.stack([t1, t2, normal], axis=2)          # columns are the axes
    covs = covariance_from_axes(frames, np.broadcast_to(np.asarray(axis_stds, np.float64), (n, 3)))
    if attr_dist == "normal":
        attrs = rng.standard_normal((n, channels))
    else:
        attrs = rng.uniform(0.0, 1.0, (n, channels))
    return Scene(means=pos.astype(np.float32), covs=covs, attrs=attrs.astype(np.float32))


def cloud_scene(rng: np.random.Generator, n: int, channels: int = 3,
                lo=(-1.0, -1.0, 2.0), hi=(1.0, 1.0, 4.0),
                std_range=(0.005, 0.1)) -> Scene:
    """Random anisotropic ellipsoid cloud: uniform centres in a box, per-axis
    standard deviations log-uniform in ``std_range``, uniform random rotations."""
    means = rng.uniform(lo, hi, (n, 3))
    stds = np.exp(rng.uniform(math.log(std_range[0]), math.log(std_range[1]), (n, 3)))
    frames = random_rotations(rng, n)
    covs = covariance_from_axes(frames, stds)
    attrs = rng.uniform(0.0, 1.0, (n, channels))
    return Scene(means=means.astype(np.float32), covs=covs, attrs=attrs.astype(np.float32))


def isotropic_scene(rng: np.random.Generator, n: int, channels: int = 3,
                    lo=(-1.0, -1.0, 2.0), hi=(1.0, 1.0, 4.0), sigma_range=(0.02, 0.08)) -> Scene:
    """Spheres: uniform centres in a box, Sigma = sigma^2 I with sigma uniform."""
    means = rng.uniform(lo, hi, (n, 3))
    sig = rng.uniform(sigma_range[0], sigma_range[1], n)
    covs = np.zeros((n, 6))
    covs[:, 0] = covs[:, 3] = covs[:, 5] = sig ** 2
    attrs = rng.uniform(0.0, 1.0, (n, channels))
    return Scene(means=means.astype(np.float32), covs=covs.astype(np.float32),
                 attrs=attrs.astype(np.float32))


def random_pose(rng: np.random.Generator, size: int, dist_range=(2.5, 4.0),
                elev_deg=(-30.0, 60.0)) -> Camera:
    """Look-at pose around the origin: azimuth U[0, 2pi), elevation and distance uniform."""
    az = rng.uniform(0.0, 2.0 * math.pi)
    el = math.radians(rng.uniform(*elev_deg))
    d = rng.uniform(*dist_range)
    pos = d * np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
    return look_at_camera(pos, size)


def multiview_cameras(n: int = 20, size: int = 128, dist: float = 3.5, focal_scale: float = 1.2,
                      elev_deg: float = 15.0) -> List[Camera]:
    """n look-at views around the origin: azimuths evenly spaced, elevation
    alternating +-elev_deg, all at distance dist (the multi-view setting of
    the shape-fitting experiment)."""
    cams = []
    for k in range(n):
        az = 2.0 * math.pi * k / n
        el = math.radians(elev_deg if k % 2 == 0 else -elev_deg)
        pos = dist * np.array([math.cos(el) * math.sin(az), math.sin(el), math.cos(el) * math.cos(az)])
        cams.append(look_at_camera(pos, size, focal=focal_scale * size))
    return cams


def bumpy_target(subdivisions: int = 5, amplitude: float = 0.4, flatten: float = 0.3) -> Scene:
    """A synthetic fitting target: an icosphere pushed out radially by
    1 + amplitude sin(3x) cos(2y) sin(2z + 1), converted to flattened
    Gaussians (zeta = 0.5), coloured by its unit normal, 0.5 + 0.5 n."""
    from .convert import icosphere, mesh_to_gaussians, vertex_normals

    v, f = icosphere(subdivisions)
    r = 1.0 + amplitude * np.sin(3 * v[:, 0]) * np.cos(2 * v[:, 1]) * np.sin(2 * v[:, 2] + 1.0)
    v = v * r[:, None]
    means, covs = mesh_to_gaussians(v, f, 0.5, flatten=flatten)
    colors = (0.5 + 0.5 * vertex_normals(v, f)).astype(np.float32)
    return Scene(means=means, covs=covs, attrs=colors)


def sphere_start(subdivisions: int = 4, radius: float = 1.0, gray: float = 0.5) -> Scene:
    """The fitting start: an icosphere (2,562 vertices at 4 subdivisions)
    converted to isotropic Gaussians (zeta = 0.5), uniform grey."""
    from .convert import icosphere, mesh_to_gaussians

    v, f = icosphere(subdivisions, radius)
    means, covs = mesh_to_gaussians(v, f, 0.5)
    return Scene(means=means, covs=covs, attrs=np.full((v.shape[0], 3), gray, np.float32))


def upstream_gradient(rng: np.random.Generator, h: int, w: int, c: int) -> np.ndarray:
    return rng.standard_normal((h, w, c)).astype(np.float32)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def config_small(seed: int = 1) -> Job:
    """64x64 pinhole image (F = 64), 512 spheres in [-1,1]^2 x [2,4], sigma in
    [0.02, 0.08], RGB in [0,1], K = 16, forward only."""
    rng = np.random.default_rng(seed)
    scene = isotropic_scene(rng, 512, 3)
    return Job(scene=scene, camera=identity_camera(64, 64.0), K=16, name="sphere512_64px_K16")


def config_torus(seed: int = 2, size: int = 512, n: int = 10_000, channels: int = 16,
                 with_grad: bool = True) -> Job:
    """512x512 image (F = 512), 10,000 flattened kernels on a torus 3 units in
    front of the camera, 16 N(0,1) channels, K = 20, N(0,1) upstream gradient."""
    rng = np.random.default_rng(seed)
    scene = torus_scene(rng, n, channels, centre=(0.0, 0.0, 3.0))
    cam = identity_camera(size, float(size))
    grad = upstream_gradient(rng, size, size, channels) if with_grad else None
    return Job(scene=scene, camera=cam, K=20, grad_image=grad, name=f"torus{n}_{size}px_C{channels}_K20")


def config_poses(seed: int = 3, n_poses: int = 256, size: int = 128, n: int = 4096) -> List[Job]:
    """One 4,096-kernel torus at the origin (3 U[0,1] channels) seen from
    ``n_poses`` look-at poses at size x size, K = 20, N(0,1) upstream gradients."""
    rng = np.random.default_rng(seed)
    scene = torus_scene(rng, n, 3, centre=(0.0, 0.0, 0.0), attr_dist="uniform")
    jobs = []
    for p in range(n_poses):
        cam = random_pose(rng, size)
        g = upstream_gradient(rng, size, size, 3)
        jobs.append(Job(scene=scene, camera=cam, K=20, grad_image=g, name=f"pose{p}"))
    return jobs


def config_uneven(seed: int = 4, n_scenes: int = 64, max_kernels: int = 100_000) -> List[Job]:
    """64 ellipsoid clouds with log-uniform kernel counts in [1e3, 1e5], image
    sizes from {64,128,256,512}, K from {8,16,32}, identity cameras."""
    rng = np.random.default_rng(seed)
    jobs = []
    for s in range(n_scenes):
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(max_kernels)))))
        size = int(rng.choice([64, 128, 256, 512]))
        k = int(rng.choice([8, 16, 32]))
        scene = cloud_scene(rng, n, 3)
        g = upstream_gradient(rng, size, size, 3)
        jobs.append(Job(scene=scene, camera=identity_camera(size), K=k, grad_image=g,
                        name=f"cloud{s}_N{n}_{size}px_K{k}"))
    return jobs


def serving_scenes(seed: int = 5, sizes=(10_000, 25_000, 50_000, 100_000, 150_000, 200_000)) -> List[Scene]:
    """Resident scenes for the request mix, alternating torus and cloud
    generators, all centred on the origin."""
    rng = np.random.default_rng(seed)
    out = []
    for idx, n in enumerate(sizes):
        if idx % 2 == 0:
            out.append(torus_scene(rng, n, 3, centre=(0.0, 0.0, 0.0), attr_dist="uniform"))
        else:
            out.append(cloud_scene(rng, n, 3, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0)))
    return out


def serving_requests(seed: int, n_requests: int, n_scenes: int,
                     sizes=(128, 256, 512, 1024), backward_fraction: float = 0.5):
    """Request descriptors: (scene id, camera, with_backward, upstream-gradient seed)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(n_requests):
        sid = int(rng.integers(n_scenes))
        size = int(rng.choice(sizes))
        cam = random_pose(rng, size)
        bwd = bool(rng.uniform() < backward_fraction)
        reqs.append(dict(scene=sid, camera=cam, backward=bwd, grad_seed=int(rng.integers(2**31))))
    return reqs
