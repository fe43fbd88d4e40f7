"""Seeded synthetic inputs: material layouts and initial velocity fields.

This module holds no arithmetic of the method (no equilibrium, collision or
streaming); it only builds the geometries and initial macroscopic fields that
both the GPU path and the test oracle are fed with.  Material numbers follow the
guide (Geometry Creation, "Setting Material Numbers"): 1 fluid, 2 no-slip
bounce-back wall, 3 moving (velocity) wall, 0 no dynamics.

Arrays are numpy, shaped (nz, ny, nx) with x fastest; velocity fields are
(3, nz, ny, nx).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

PERIODIC_X, PERIODIC_Y, PERIODIC_Z = 1, 2, 4


@dataclass
class Workload:
    name: str
    descriptor: int          # 0 = D2Q9, 1 = D3Q19
    shape: tuple             # (nx, ny, nz)
    tau: float
    material: np.ndarray     # uint8 (nz, ny, nx)
    periodic: int
    u0: np.ndarray | None = None   # (3, nz, ny, nx) initial velocity or None
    g: tuple = (0.0, 0.0, 0.0)
    u_wall: tuple = (0.0, 0.0, 0.0)
    steps: int = 0
    storage: str = "f32"


def cavity2d(n=64, u_lid=0.05, tau=0.6, steps=2000):
    """Lid-driven cavity on an n x n node grid: the outer ring is a resting
    bounce-back wall and the whole top row (corners included) is the lid."""
    mat = np.full((1, n, n), 2, np.uint8)
    mat[0, 1:-1, 1:-1] = 1
    mat[0, -1, :] = 3
    return Workload("cavity2d", 0, (n, n, 1), tau, mat, 0, None, (0.0, 0.0, 0.0),
                    (u_lid, 0.0, 0.0), steps, "f64")


def tgv3d_velocity(nx, ny, nz, u0, kx=None, ky=None, kz=None):
    """Taylor-Green initial field u = u0 sin(kx x) cos(ky y) cos(kz z),
    v = -u0 (kx/ky) cos(kx x) sin(ky y) cos(kz z), w = 0 (divergence free);
    k defaults to one period per box edge."""
    kx = 2 * math.pi / nx if kx is None else kx
    ky = 2 * math.pi / ny if ky is None else ky
    kz = 2 * math.pi / nz if kz is None else kz
    x, y, z = np.arange(nx), np.arange(ny), np.arange(nz)
    sx, cx = np.sin(kx * x)[None, None, :], np.cos(kx * x)[None, None, :]
    sy, cy = np.sin(ky * y)[None, :, None], np.cos(ky * y)[None, :, None]
    cz = np.cos(kz * z)[:, None, None]
    u = np.zeros((3, nz, ny, nx))
    u[0] = u0 * (sx * cy) * cz
    u[1] = -u0 * (kx / ky) * (cx * sy) * cz
    return u


def tgv3d(n=256, u0=0.05, tau=0.8, steps=1000, storage="f32", with_field=True):
    """Fully periodic Taylor-Green vortex on an n^3 lattice (D3Q19)."""
    mat = np.ones((n, n, n), np.uint8)
    u = tgv3d_velocity(n, n, n, u0) if with_field else None
    return Workload("tgv3d", 1, (n, n, n), tau, mat, 7, u, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0),
                    steps, storage)


def tgv_ensemble(count=256, seed=1107, lmin=16, lmax=96, u0_range=(0.01, 0.08),
                 tau_range=(0.55, 1.0)):
    """Ensemble of periodic D3Q19 Taylor-Green lattices: every edge length
    log-uniform in [lmin, lmax] (independently per axis, so boxes are not
    cubic), u0 uniform in u0_range, tau uniform in tau_range.  Returns
    (shapes [(nx, ny, nz)], u0 [count], tau [count]); the initial field of
    member l is tgv3d_velocity(*shapes[l], u0[l])."""
    rng = np.random.default_rng(seed)
    lo, hi = math.log(lmin), math.log(lmax)
    shapes = [tuple(int(round(math.exp(v))) for v in rng.uniform(lo, hi, 3)) for _ in range(count)]
    u0 = rng.uniform(*u0_range, count)
    tau = rng.uniform(*tau_range, count)
    return shapes, u0, tau


def porous_channel(nx=128, ny=64, nz=64, seed=4668, sigma=4.0):
    """Channel for porosity gradients: periodic along x, resting walls on the
    outer y and z layers, porosity = seeded white noise smoothed by a Gaussian
    of sigma cells (periodic along x), min-max mapped to [0, 1].
    Returns (material (nz, ny, nx) uint8, porosity (nz, ny, nx) float64)."""
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    mat = np.ones((nz, ny, nx), np.uint8)
    mat[:, 0, :] = 2
    mat[:, -1, :] = 2
    mat[0, :, :] = 2
    mat[-1, :, :] = 2
    noise = rng.standard_normal((nz, ny, nx))
    smooth = gaussian_filter(noise, sigma, mode=("nearest", "nearest", "wrap"))
    por = (smooth - smooth.min()) / (smooth.max() - smooth.min())
    return mat, por


def channel_spheres(nx=512, ny=128, nz=128, seed=2307, solid_fraction=0.20, rmin=4.0,
                    rmax=10.0, g=1e-6, tau=0.7, steps=5000, storage="f32"):
    """Body-force-driven channel: periodic along x, resting walls on the outer y
    and z layers, random overlapping solid spheres (radius uniform in
    [rmin, rmax], centre uniform in the box, minimum image along x) added until
    the solid fraction of the interior reaches solid_fraction."""
    rng = np.random.default_rng(seed)
    mat = np.ones((nz, ny, nx), np.uint8)
    mat[:, 0, :] = 2
    mat[:, -1, :] = 2
    mat[0, :, :] = 2
    mat[-1, :, :] = 2
    interior = (nz - 2) * (ny - 2) * nx
    solid = 0
    while solid < solid_fraction * interior:
        cx, cy, cz = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz)
        r = rng.uniform(rmin, rmax)
        ri = int(math.ceil(r))
        xs = np.arange(int(math.floor(cx)) - ri, int(math.floor(cx)) + ri + 2)
        ys = np.arange(max(1, int(math.floor(cy)) - ri), min(ny - 1, int(math.floor(cy)) + ri + 2))
        zs = np.arange(max(1, int(math.floor(cz)) - ri), min(nz - 1, int(math.floor(cz)) + ri + 2))
        if ys.size == 0 or zs.size == 0:
            continue
        dx = xs - cx
        dx = dx - nx * np.round(dx / nx)
        Z, Y, X = np.meshgrid(zs - cz, ys - cy, dx, indexing="ij")
        inside = X * X + Y * Y + Z * Z <= r * r
        sub = mat[np.ix_(zs, ys, xs % nx)]
        newly = inside & (sub == 1)
        solid += int(newly.sum())
        sub[inside] = 2
        mat[np.ix_(zs, ys, xs % nx)] = sub
    return Workload("channel_spheres", 1, (nx, ny, nz), tau, mat, PERIODIC_X, None,
                    (g, 0.0, 0.0), (0.0, 0.0, 0.0), steps, storage)


def random_geometry(descriptor, shape, periodic, seed, wall_fraction=0.15, moving_top=True):
    """Small random layout for parity tests: walls on the faces of every
    non-periodic axis (the top y face moving when moving_top), plus randomly
    scattered interior wall cells, some of them moving."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    mat = np.ones((nz, ny, nx), np.uint8)
    interior = rng.uniform(size=mat.shape) < wall_fraction
    mat[interior] = np.where(rng.uniform(size=int(interior.sum())) < 0.25, 3, 2)
    if not periodic & PERIODIC_X:
        mat[:, :, 0] = 2
        mat[:, :, -1] = 2
    if not periodic & PERIODIC_Y:
        mat[:, 0, :] = 2
        mat[:, -1, :] = 3 if moving_top else 2
    if descriptor == 1 and not periodic & PERIODIC_Z:
        mat[0, :, :] = 2
        mat[-1, :, :] = 2
    return mat


def random_velocity(shape, seed, amplitude=0.05, dim=3):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    u = np.zeros((3, nz, ny, nx))
    u[:dim] = rng.uniform(-amplitude, amplitude, (dim, nz, ny, nx))
    return u


def random_density(shape, seed, amplitude=0.02):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    return 1.0 + rng.uniform(-amplitude, amplitude, (nz, ny, nx))
