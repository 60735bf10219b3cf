"""Closed-form prism sensitivities and the dense sensitivity matrix (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper (Sec. 2.1, eq. d=gm) builds A^(1) from the vertical gravity of a right
rectangular prism (Haaz) and A^(2) from the total-field anomaly of a prism with
induced magnetisation only (Rao & Babu), without printing either formula.  This
module writes both out from their definitions:

* gravity:   g_z = G rho * int_V Z / R^3 dV, with (X, Y, Z) = source - station,
  z positive down.  Its exact antiderivative, summed over the 8 corners with sign
  (-1)^(i+j+k), is  Z atan(XY/(ZR)) - X ln(Y+R) - Y ln(X+R).
* magnetic:  Delta T = (F / 4 pi) f^T H f per SI unit of susceptibility, with
  f = (cos I sin D, cos I cos D, sin I) in (East, North, Down) and H the Hessian
  of int_V dV/R:  H_xx = -sum mu atan(YZ/(XR)), H_yy = -sum mu atan(XZ/(YR)),
  H_zz = -sum mu atan(XY/(ZR)), H_xy = sum mu ln(Z+R), H_xz = sum mu ln(Y+R),
  H_yz = sum mu ln(X+R).

Geometry (the paper fixes only that stations sit at prism centres on the surface,
Sec. 2.7.1): x = East (station index p, prism index a), y = North (q, b),
z = down; prism (a, b, r) spans [a dx,(a+1)dx] x [b dy,(b+1)dy] x
[top + r dz, top + (r+1) dz]; station (p, q) sits at ((p+ox+1/2)dx, (q+oy+1/2)dy, -h),
above the centre of prism column (p+ox, q+oy).  ox = oy = 0 with sx = nx, sy = ny is the
paper's layout; a station grid over an interior part of a larger (padded) model domain
(Sec. 2.7.1) has sx < nx and an offset.

Units: density in g/cc and gravity in mGal (C_G = 6.6743e-11 * 1e3 * 1e5), field
and anomaly in nT, susceptibility in SI.

Pins (tests/test_oracle_prism.py): Gauss-Legendre cubature of the defining
integrands, additivity over sub-prisms, the point-mass and dipole far-field limits,
Laplace (tr H = 0), Poisson's relation H_zz = -d(g_z/C_G)/dh, mirror symmetries,
the Bouguer slab limit and BTTB shift invariance of the dense matrix.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

C_G = 6.6743e-11 * 1.0e3 * 1.0e5   # mGal per (g/cc * m)
GRAVITY = 0
MAGNETIC = 1


@dataclass(frozen=True)
class Geometry:
    """Station grid sx x sy over a prism grid nx x ny x nz (Sec. 2.7.1)."""
    sx: int
    sy: int
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    h: float = 1.0          # station height above the top surface (m)
    top: float = 0.0        # depth of the top of layer 0 (m)
    incl: float = 65.0      # inducing field inclination (deg)
    decl: float = 2.0       # inducing field declination (deg)
    field: float = 50000.0  # inducing field intensity (nT)
    ox: int = 0             # prism column under station column 0
    oy: int = 0             # prism row under station row 0

    @property
    def m(self) -> int:
        return self.sx * self.sy

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


def _ln_sum(a, R, b, c):
    """ln(a + R) with R = sqrt(a^2+b^2+c^2), rewritten as ln((b^2+c^2)/(R-a)) for a < 0
    so that the cancellation a + R ~ 0 never happens."""
    a = np.asarray(a, dtype=np.float64)
    pos = np.log(np.where(a >= 0, a + R, 1.0))
    neg = np.log(np.where(a < 0, (b * b + c * c) / np.where(a < 0, R - a, 1.0), 1.0))
    return np.where(a >= 0, pos, neg)


def _corners(x0, y0, z0, xb, yb, zb):
    """Relative corner coordinates X_i = x_i - x0 etc., with the corner sign mu."""
    out = []
    for i in (0, 1):
        for j in (0, 1):
            for k in (0, 1):
                mu = (-1.0) ** (i + j + k + 3)      # (-1)^(i+j+k) with 1-based indices
                out.append((mu, xb[i] - x0, yb[j] - y0, zb[k] - z0))
    return out


def gravity_prism(x0, y0, z0, xb, yb, zb):
    """Vertical gravity (mGal) at (x0, y0, z0) of a 1 g/cc prism xb x yb x zb (z down)."""
    acc = 0.0
    for mu, X, Y, Z in _corners(x0, y0, z0, xb, yb, zb):
        R = np.sqrt(X * X + Y * Y + Z * Z)
        F = Z * np.arctan(X * Y / (Z * R)) - X * _ln_sum(Y, R, X, Z) - Y * _ln_sum(X, R, Y, Z)
        acc = acc + mu * F
    return C_G * acc


def prism_hessian(x0, y0, z0, xb, yb, zb):
    """Hessian H_ab = d^2/da db of int_V dV/R (dimensionless), as a dict of 6 entries."""
    H = dict(xx=0.0, yy=0.0, zz=0.0, xy=0.0, xz=0.0, yz=0.0)
    for mu, X, Y, Z in _corners(x0, y0, z0, xb, yb, zb):
        R = np.sqrt(X * X + Y * Y + Z * Z)
        H["xx"] = H["xx"] - mu * np.arctan(Y * Z / (X * R))
        H["yy"] = H["yy"] - mu * np.arctan(X * Z / (Y * R))
        H["zz"] = H["zz"] - mu * np.arctan(X * Y / (Z * R))
        H["xy"] = H["xy"] + mu * _ln_sum(Z, R, X, Y)
        H["xz"] = H["xz"] + mu * _ln_sum(Y, R, X, Z)
        H["yz"] = H["yz"] + mu * _ln_sum(X, R, Y, Z)
    return H


def field_direction(incl_deg: float, decl_deg: float):
    """Unit vector of the inducing field in (East, North, Down)."""
    I = np.deg2rad(incl_deg)
    D = np.deg2rad(decl_deg)
    return np.array([np.cos(I) * np.sin(D), np.cos(I) * np.cos(D), np.sin(I)])


def magnetic_prism(x0, y0, z0, xb, yb, zb, incl_deg, decl_deg, field_nt):
    """Total-field anomaly (nT) at (x0, y0, z0) of a prism of unit SI susceptibility
    magnetised by induction along the main field (no remanence, no demagnetisation)."""
    f = field_direction(incl_deg, decl_deg)
    H = prism_hessian(x0, y0, z0, xb, yb, zb)
    q = (f[0] * f[0] * H["xx"] + f[1] * f[1] * H["yy"] + f[2] * f[2] * H["zz"]
         + 2.0 * f[0] * f[1] * H["xy"] + 2.0 * f[0] * f[2] * H["xz"]
         + 2.0 * f[1] * f[2] * H["yz"])
    return field_nt / (4.0 * np.pi) * q


def station_xyz(g: Geometry, p, q):
    return (np.asarray(p) + g.ox + 0.5) * g.dx, (np.asarray(q) + g.oy + 0.5) * g.dy, -g.h


def prism_bounds(g: Geometry, a, b, r):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    xb = (a * g.dx, (a + 1.0) * g.dx)
    yb = (b * g.dy, (b + 1.0) * g.dy)
    zb = (g.top + r * g.dz, g.top + (r + 1.0) * g.dz)
    return xb, yb, zb


def sensitivity(kind: int, g: Geometry, p, q, a, b, r):
    """Entry of A for station (p, q) and prism (a, b, r); arrays broadcast."""
    x0, y0, z0 = station_xyz(g, p, q)
    xb, yb, zb = prism_bounds(g, a, b, r)
    if kind == GRAVITY:
        return gravity_prism(x0, y0, z0, xb, yb, zb)
    return magnetic_prism(x0, y0, z0, xb, yb, zb, g.incl, g.decl, g.field)


def dense_matrix(kind: int, g: Geometry) -> np.ndarray:
    """Dense A (m x n), rows ordered (p, q) with q fastest, columns ordered (r, a, b)
    with b fastest, i.e. blocked by depth layer as in Sec. 2.7.1.  Every entry is
    evaluated from absolute station and prism coordinates."""
    p, q = np.meshgrid(np.arange(g.sx), np.arange(g.sy), indexing="ij")
    r, a, b = np.meshgrid(np.arange(g.nz), np.arange(g.nx), np.arange(g.ny), indexing="ij")
    P = p.reshape(-1, 1)
    Q = q.reshape(-1, 1)
    R = r.reshape(1, -1)
    Acol = a.reshape(1, -1)
    B = b.reshape(1, -1)
    return np.asarray(sensitivity(kind, g, P, Q, Acol, B, R), dtype=np.float64)


def dense_matvec(A: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = A m with m shaped [nz][nx][ny]; returns [sx*sy] (eq. d=gm)."""
    return A @ x.reshape(-1)


def dense_rmatvec(A: np.ndarray, r: np.ndarray) -> np.ndarray:
    """z = A^T r with r shaped [sx][sy]; returns [nz*nx*ny]."""
    return A.T @ r.reshape(-1)
