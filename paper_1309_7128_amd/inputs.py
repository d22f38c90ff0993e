"""Seeded synthetic workloads for the pressure-Poisson solve.

This module only draws random numbers and evaluates closed-form velocity fields on the
staggered (MAC) grid.  It holds none of the solver's arithmetic: the right-hand side of a
solve is the discrete divergence of these fields, and each side (the HIP library and the
CPU oracle) computes that divergence itself.

The paper's benchmark flows (a shear-driven cavity, Sec. 4.3.1, and a turbulent jet,
Sec. 4.3.2) are time histories of a Navier-Stokes solver that is not part of this library.
The recipes below stand in for their shapes: broadband random faces, a smooth Fourier field
with white noise on top, and a tanh jet with a k^(-5/3) perturbation.

Layout (row-major, cell (j, i) is row j, column i, 0-based, i along x):
  u: x-face velocities, shape (ny, nx + 1), face i is the west face of cell i;
     periodic in x: shape (ny, nx), face 0 doubles as face nx.
  v: y-face velocities, shape (ny + 1, nx), face j is the south face of cell j.
All arrays are float64 and C-contiguous.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

NEUMANN = "neumann"
PERIODIC = "periodic"


@dataclasses.dataclass(frozen=True)
class Workload:
    """Grid, boundary conditions and solver settings of one synthetic workload."""

    name: str
    nx: int
    ny: int
    batch: int
    lx: float
    ly: float
    bc_x: str
    bc_y: str
    coarsen: int
    precision: str  # "fp64" or "mixed"
    rtol: float

    @property
    def h(self) -> float:
        return self.lx / self.nx

    @property
    def u_shape(self):
        return (self.ny, self.nx) if self.bc_x == PERIODIC else (self.ny, self.nx + 1)

    @property
    def v_shape(self):
        return (self.ny + 1, self.nx)


# The five workloads.  Sizes, boundary conditions, coarsening and tolerance follow the
# problem statement (grid size, tile size, boundary conditions and tolerance are the
# parameters the paper's solver exposes, Sec. 4.1 and Sec. 4.3.1).
WORKLOADS = {
    "cavity256_fp64": Workload("cavity256_fp64", 256, 256, 1, 1.0, 1.0, NEUMANN, NEUMANN, 16, "fp64", 1e-10),
    "cavity2048_fp64": Workload("cavity2048_fp64", 2048, 2048, 1, 1.0, 1.0, NEUMANN, NEUMANN, 16, "fp64", 1e-10),
    "cavity8192_mixed": Workload("cavity8192_mixed", 8192, 8192, 1, 1.0, 1.0, NEUMANN, NEUMANN, 32, "mixed", 1e-10),
    "jet4096x8192_mixed": Workload("jet4096x8192_mixed", 4096, 8192, 1, 0.5, 1.0, PERIODIC, NEUMANN, 16, "mixed", 1e-8),
    "batch8x1024_mixed": Workload("batch8x1024_mixed", 1024, 1024, 8, 1.0, 1.0, NEUMANN, NEUMANN, 16, "mixed", 1e-10),
}


def uniform_faces(seed: int, nx: int, ny: int, bc_x: str = NEUMANN):
    """Every face velocity drawn from U[-1, 1]: u first, then v, row-major."""
    rng = np.random.default_rng(seed)
    ushape = (ny, nx) if bc_x == PERIODIC else (ny, nx + 1)
    u = rng.uniform(-1.0, 1.0, size=ushape)
    v = rng.uniform(-1.0, 1.0, size=(ny + 1, nx))
    return np.ascontiguousarray(u), np.ascontiguousarray(v)


def _draw_smooth_modes(rng, count=64, kmax=32):
    """Integer wave vectors uniform in [-kmax, kmax]^2 without (0, 0), kept if |k| <= kmax."""
    modes = []
    while len(modes) < count:
        kx, ky = (int(t) for t in rng.integers(-kmax, kmax + 1, size=2))
        if (kx, ky) != (0, 0) and kx * kx + ky * ky <= kmax * kmax:
            modes.append((kx, ky))
    return np.array(modes, dtype=np.float64)


def _mode_sum(xs, ys, kx, ky, coef, lx, ly):
    """sum_m Re(coef_m * exp(2 pi i (kx_m x / lx + ky_m y / ly))) on the tensor grid ys x xs.

    Evaluated separably as a (len(ys) x M) @ (M x len(xs)) complex product so that
    8192^2 grids take seconds."""
    ey = np.exp(2j * np.pi * np.outer(ys / ly, ky)) * coef[None, :]
    ex = np.exp(2j * np.pi * np.outer(kx, xs / lx))
    return np.ascontiguousarray((ey @ ex).real)


def smooth64(seed: int, nx: int, ny: int, lx: float = 1.0, ly: float = 1.0,
             noise_sigma: float = 1e-3, noise_on: str = "velocity"):
    """Smooth field: 64 random Fourier modes with |k| <= 32 and amplitude |k|^-2, plus noise.

    Draw order: the 64 wave vectors, 64 phases for u, 64 phases for v, then Gaussian noise
    (sigma = noise_sigma) on every u face, then on every v face.  With noise_on="rhs" no
    face noise is drawn; the caller adds noise to the divergence instead (draw it from
    `rhs_noise`)."""
    rng = np.random.default_rng(seed)
    k = _draw_smooth_modes(rng)
    amp = 1.0 / (k[:, 0] ** 2 + k[:, 1] ** 2)
    phu = rng.uniform(0.0, 2.0 * np.pi, size=len(k))
    phv = rng.uniform(0.0, 2.0 * np.pi, size=len(k))
    h = lx / nx
    xu = np.arange(nx + 1) * h
    yu = (np.arange(ny) + 0.5) * h
    xv = (np.arange(nx) + 0.5) * h
    yv = np.arange(ny + 1) * h
    u = _mode_sum(xu, yu, k[:, 0], k[:, 1], amp * np.exp(1j * phu), lx, ly)
    v = _mode_sum(xv, yv, k[:, 0], k[:, 1], amp * np.exp(1j * phv), lx, ly)
    if noise_on == "velocity" and noise_sigma > 0:
        u += rng.normal(0.0, noise_sigma, size=u.shape)
        v += rng.normal(0.0, noise_sigma, size=v.shape)
    return u, v


def jet(seed: int, nx: int = 4096, ny: int = 8192, lx: float = 0.5, ly: float = 1.0,
        step: int = 0, n_modes: int = 256, rms: float = 0.05):
    """Jet along x (periodic in x, walls in y) with an isotropic k^(-5/3) perturbation.

    Base flow: u = (tanh((y - yc + W/2)/d) - tanh((y - yc - W/2)/d)) / 2 with W = ly/16,
    d = W/8, yc = ly/2 (peak speed 1), v = 0; it is exactly divergence-free.
    Perturbation: n_modes integer wave vectors (mx, my) with physical wavenumber
    |k| = 2 pi sqrt((mx/lx)^2 + (my/ly)^2) in [2 pi/lx, 256 * 2 pi/lx] (rejection sampled
    uniformly on the integer box), amplitude |k|^(-4/3) (energy spectrum k^(-5/3) in 2D),
    a random phase and a random unit direction (cos t, sin t) for (u, v), scaled so the
    perturbation's rms over all faces is `rms`.  Step t shifts the perturbation by t cells
    in +x.  v on the two wall rows is zero.
    Draw order: wave vectors, phases, directions."""
    rng = np.random.default_rng(seed)
    mxmax = 256
    mymax = int(256 * ly / lx)
    modes = []
    while len(modes) < n_modes:
        mx = int(rng.integers(-mxmax, mxmax + 1))
        my = int(rng.integers(-mymax, mymax + 1))
        q = (mx / lx) ** 2 + (my / ly) ** 2
        if (1.0 / lx) ** 2 <= q <= (256.0 / lx) ** 2:
            modes.append((mx, my))
    m = np.array(modes, dtype=np.float64)
    kmag = 2.0 * np.pi * np.sqrt((m[:, 0] / lx) ** 2 + (m[:, 1] / ly) ** 2)
    amp = kmag ** (-4.0 / 3.0)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    th = rng.uniform(0.0, 2.0 * np.pi, size=n_modes)
    h = lx / nx
    shift = step * h
    xu = np.arange(nx) * h - shift
    yu = (np.arange(ny) + 0.5) * h
    xv = (np.arange(nx) + 0.5) * h - shift
    yv = np.arange(ny + 1) * h
    up = _mode_sum(xu, yu, m[:, 0], m[:, 1], amp * np.cos(th) * np.exp(1j * ph), lx, ly)
    vp = _mode_sum(xv, yv, m[:, 0], m[:, 1], amp * np.sin(th) * np.exp(1j * ph), lx, ly)
    vp[0, :] = 0.0
    vp[-1, :] = 0.0
    cnt = up.size + vp.size
    scale = rms / math.sqrt((np.sum(up * up) + np.sum(vp * vp)) / cnt)
    up *= scale
    vp *= scale
    yc = 0.5 * ly
    w = ly / 16.0
    d = w / 8.0
    base = 0.5 * (np.tanh((yu - yc + 0.5 * w) / d) - np.tanh((yu - yc - 0.5 * w) / d))
    u = up + base[:, None]
    return np.ascontiguousarray(u), np.ascontiguousarray(vp)


def normal_faces(seed: int, ushape, vshape):
    """Loss weights w ~ N(0, 1) on every face: u faces first, then v faces."""
    rng = np.random.default_rng(seed)
    return rng.normal(size=ushape), rng.normal(size=vshape)


def rhs_noise(seed: int, shape, sigma: float):
    """Gaussian noise for a right-hand side (the noise_on="rhs" reading)."""
    return np.random.default_rng(seed).normal(0.0, sigma, size=shape)


def workload_fields(name: str, batch_index: int = 0, step: int = 0):
    """Face velocities (u, v) of one grid of a named workload."""
    w = WORKLOADS[name]
    if name == "cavity256_fp64":
        return uniform_faces(1, w.nx, w.ny)
    if name == "cavity2048_fp64":
        return smooth64(2, w.nx, w.ny)
    if name == "cavity8192_mixed":
        return smooth64(3, w.nx, w.ny)
    if name == "jet4096x8192_mixed":
        return jet(4, w.nx, w.ny, w.lx, w.ly, step=step)
    if name == "batch8x1024_mixed":
        return smooth64(500 + batch_index, w.nx, w.ny)
    raise KeyError(name)


def batch_weights(batch_index: int, ushape, vshape):
    """Loss weights of grid b of the batched projection workload (seed 600 + b)."""
    return normal_faces(600 + batch_index, ushape, vshape)
