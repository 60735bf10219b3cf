"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the inversion method: it only draws models,
noise and sizes with ``numpy.random.default_rng`` and states the geometry of each
workload as plain numbers.  Both the HIP path and the oracle consume what it
returns; neither imports the other.

Seeds are ``1000 * workload + index``.  The paper's own synthetic bodies exist only
as figures and its field data are not available, so every workload below is a
stand-in with the paper's sizes, contrasts, noise model and parameters.
"""
from __future__ import annotations

from dataclasses import dataclass, asdict
from typing import List, Tuple

import numpy as np


@dataclass(frozen=True)
class Grid:
    """Stations sx x sy over prisms nx x ny x nz; station (p, q) sits above the centre of
    prism column (p + ox, q + oy)."""
    sx: int
    sy: int
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    h: float = 1.0
    top: float = 0.0
    incl: float = 65.0
    decl: float = 2.0
    field: float = 50000.0
    ox: int = 0
    oy: int = 0

    def asdict(self):
        return asdict(self)

    @property
    def model_shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.nx, self.ny)

    @property
    def data_shape(self) -> Tuple[int, int]:
        return (self.sx, self.sy)


# 16x16 stations over 16x16x8 prisms of 50 m cubes (BCCB 31 -> 32).
SMALL = Grid(16, 16, 16, 16, 8, 50.0, 50.0, 50.0)
# 12x12x6 subcase (BCCB 23 -> 24, a radix-3 size).
SUB = Grid(12, 12, 12, 12, 6, 50.0, 50.0, 50.0)
# 128x128 over 128x128x20, 40 x 40 x 25 m cells.
MID = Grid(128, 128, 128, 128, 20, 40.0, 40.0, 25.0)
# 256x256 over 256x256x32, 40 x 40 x 25 m cells (the large single-GPU workload).
LARGE = Grid(256, 256, 256, 256, 32, 40.0, 40.0, 25.0)
# batch of models on 128x128x24 prisms.
BATCH = Grid(128, 128, 128, 128, 24, 40.0, 40.0, 25.0)


def rng(workload: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng(1000 * workload + index)


def uniform_models(g: Grid, seed_workload: int = 1, index: int = 0):
    """Density U[0,1] g/cc and susceptibility U[0,0.05] SI, iid per prism."""
    r = rng(seed_workload, index)
    rho = r.uniform(0.0, 1.0, g.model_shape)
    kap = r.uniform(0.0, 0.05, g.model_shape)
    return rho, kap


def random_boxes(g: Grid, nbodies: int = 3, seed_workload: int = 2, index: int = 0):
    """nbodies rectangular bodies in a zero background: extents U{8..40} cells in x
    and y (clipped to the grid), U{2..10} layers; density U[0.2,0.6] g/cc and a
    positively correlated susceptibility 0.01 + 0.04 (rho - 0.2)/0.4 SI.  Later
    bodies overwrite earlier ones."""
    r = rng(seed_workload, index)
    rho = np.zeros(g.model_shape)
    kap = np.zeros(g.model_shape)
    for _ in range(nbodies):
        ex = int(min(r.integers(8, 41), g.nx))
        ey = int(min(r.integers(8, 41), g.ny))
        ez = int(min(r.integers(2, 11), g.nz))
        x0 = int(r.integers(0, g.nx - ex + 1))
        y0 = int(r.integers(0, g.ny - ey + 1))
        z0 = int(r.integers(0, g.nz - ez + 1))
        d = r.uniform(0.2, 0.6)
        rho[z0:z0 + ez, x0:x0 + ex, y0:y0 + ey] = d
        kap[z0:z0 + ez, x0:x0 + ex, y0:y0 + ey] = 0.01 + 0.04 * (d - 0.2) / 0.4
    return rho, kap


def dyke_and_block(g: Grid):
    """Dyke: 3 cells wide, 160 cells long (North), dipping 70 degrees (shifting
    dz cot70 / dx cells East per layer), layers 2..28; block: 48 x 32 cells, layers
    8..20.  Contrast 1 g/cc and 0.1 SI (the paper's contrasts).  Scaled to the grid
    when it is smaller than 256 x 256 x 32."""
    rho = np.zeros(g.model_shape)
    sx = g.nx / 256.0
    sy = g.ny / 256.0
    sz = g.nz / 32.0
    shift = g.dz / np.tan(np.deg2rad(70.0)) / g.dx
    x_top = int(round(60 * sx))
    y0 = int(round(48 * sy))
    y1 = min(g.ny, y0 + max(1, int(round(160 * sy))))
    for r in range(max(0, int(round(2 * sz))), min(g.nz, int(round(29 * sz)))):
        xa = x_top + int(round((r - 2 * sz) * shift))
        rho[r, max(0, xa):min(g.nx, xa + max(1, int(round(3 * sx)))), y0:y1] = 1.0
    bx0 = int(round(150 * sx))
    by0 = int(round(120 * sy))
    rho[int(round(8 * sz)):int(round(21 * sz)),
        bx0:min(g.nx, bx0 + max(1, int(round(48 * sx)))),
        by0:min(g.ny, by0 + max(1, int(round(32 * sy))))] = 1.0
    kap = 0.1 * rho
    return rho, kap


def normal_like(shape, seed_workload: int, index: int):
    """Standard normal draws (noise realisations, rough residuals)."""
    return rng(seed_workload, index).standard_normal(shape)


def noise_sigma(d: np.ndarray, tau1: float, floor: float) -> np.ndarray:
    """sigma_j = tau1 |d_j| + floor (the paper's noise model with an absolute floor:
    floor = tau2 max|d| in the paper's experiments, 0.02 mGal or 1 nT here)."""
    return tau1 * np.abs(d) + floor


def depth_weight(g: Grid, beta: float) -> np.ndarray:
    """Li-Oldenburg style depth weight (z_c + h)^(-beta/2), z_c the cell-centre depth,
    broadcast to [nz][nx][ny]; beta = 2 for gravity, 3 for magnetics."""
    zc = g.top + (np.arange(g.nz) + 0.5) * g.dz
    w = (zc + g.h) ** (-beta / 2.0)
    return np.broadcast_to(w[:, None, None], g.model_shape).copy()


def uneven_sizes(count: int = 16, seed_workload: int = 5) -> List[Grid]:
    """count independent problems: n = nx = ny ~ U{64..320}, nz ~ U{16..40}, sx = nx,
    40 x 40 x 25 m cells."""
    r = rng(seed_workload, 0)
    out = []
    for _ in range(count):
        n = int(r.integers(64, 321))
        nz = int(r.integers(16, 41))
        out.append(Grid(n, n, n, n, nz, 40.0, 40.0, 25.0))
    return out
