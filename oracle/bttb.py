"""BTTB kernel arrays and FFT2 products (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sec. 2.7.1: A = [A_(1) ... A_(nz)] by depth layer, A x = sum_r A_(r) x_(r); each
block is BTTB, A_(r)[(p,q),(a,b)] = K_r(p-a, q-b), so it is fixed by the
(sx+nx-1) x (sy+ny-1) distinct values K_r(u, v), u in [-(nx-1), sx-1],
v in [-(ny-1), sy-1], gathered in the array T_(r).

Array convention (the one ``bttb_setup`` takes): T[r][i][j] = K_r(i-(nx-1), j-(ny-1)).

The products follow the paper's FFT2 formulas on the unpadded
(sx+nx-1) x (sy+ny-1) domain (the paper's own transform size, Sec. 3.2):
  forward   A_(r) x_(r)   = IFFT2(FFT2(T_c) . FFT2(X))[0:sx, 0:sy]
  transpose A_(r)^T v     = IFFT2(conj(FFT2(T_c)) . FFT2(V))[0:nx, 0:ny]
where T_c is T placed on the circle (T_c[u mod Lx][v mod Ly] = K_r(u, v)) and X, V
are the layer / data embedded in the upper-left corner of a zero array.  The
weighted products are eq. (matrixvector): A~ x = W_d . (A (W^-1 . x)),
A~^T y = W^-1 . (A^T (W_d . y)).

Pins: these products equal the dense products of ``oracle.prism`` on small grids
(tests/test_oracle_bttb.py), which in turn are pinned by closed forms.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import prism


def kernel_array(kind: int, g: prism.Geometry) -> np.ndarray:
    """T[r][i][j] = K_r(u, v), u = i-(nx-1), v = j-(ny-1): station index minus prism index."""
    u = np.arange(-(g.nx - 1), g.sx).reshape(-1, 1)
    v = np.arange(-(g.ny - 1), g.sy).reshape(1, -1)
    T = np.empty((g.nz, u.shape[0], v.shape[1]))
    for r in range(g.nz):
        # station (u, v) over prism (0, 0, r)
        T[r] = prism.sensitivity(kind, g, u, v, 0, 0, r)
    return T


def _circular(Tr: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """Move K(u, v) from T[u+(nx-1)][v+(ny-1)] to T_c[u mod Lx][v mod Ly]."""
    return np.roll(Tr, shift=(-(nx - 1), -(ny - 1)), axis=(0, 1))


def _dims(T: np.ndarray, sx: int, sy: int):
    nz, Lx, Ly = T.shape
    return nz, Lx, Ly, Lx - sx + 1, Ly - sy + 1


def fft_matvec(T: np.ndarray, x: np.ndarray, sx: int, sy: int, workers: int = 1) -> np.ndarray:
    """y = sum_r A_(r) x_(r) via FFT2; x is [nz][nx][ny], returns [sx][sy]."""
    nz, Lx, Ly, nx, ny = _dims(T, sx, sy)
    y = np.zeros((sx, sy))
    for r in range(nz):
        Tc = _circular(T[r], nx, ny)
        X = np.zeros((Lx, Ly))
        X[:nx, :ny] = x[r]
        prod = sfft.ifft2(sfft.fft2(Tc, workers=workers) * sfft.fft2(X, workers=workers),
                          workers=workers)
        y += prod.real[:sx, :sy]
    return y


def fft_rmatvec(T: np.ndarray, v: np.ndarray, sx: int, sy: int, workers: int = 1) -> np.ndarray:
    """z_(r) = A_(r)^T v via FFT2 with conj(FFT2(T)); v is [sx][sy], returns [nz][nx][ny]."""
    nz, Lx, Ly, nx, ny = _dims(T, sx, sy)
    V = np.zeros((Lx, Ly))
    V[:sx, :sy] = v
    FV = sfft.fft2(V, workers=workers)
    z = np.empty((nz, nx, ny))
    for r in range(nz):
        Tc = _circular(T[r], nx, ny)
        prod = sfft.ifft2(np.conj(sfft.fft2(Tc, workers=workers)) * FV, workers=workers)
        z[r] = prod.real[:nx, :ny]
    return z


def weighted_matvec(T, x, winv, wd, sx, sy, workers=1):
    """A~ x = W_d . (A (W^-1 . x))  (eq. matrixvector)."""
    return wd * fft_matvec(T, winv * x, sx, sy, workers)


def weighted_rmatvec(T, v, winv, wd, sx, sy, workers=1):
    """A~^T v = W^-1 . (A^T (W_d . v))."""
    return winv * fft_rmatvec(T, wd * v, sx, sy, workers)


class FFTOperator:
    """The oracle's operator for one data set, backed by the FFT2 products."""

    def __init__(self, T: np.ndarray, sx: int, sy: int, workers: int = 1):
        self.T = np.asarray(T, dtype=np.float64)
        self.sx, self.sy = sx, sy
        self.nz, Lx, Ly, self.nx, self.ny = _dims(self.T, sx, sy)
        self.workers = workers

    def matvec(self, x):
        return fft_matvec(self.T, x, self.sx, self.sy, self.workers)

    def rmatvec(self, v):
        return fft_rmatvec(self.T, v, self.sx, self.sy, self.workers)


class DenseOperator:
    """The oracle's operator for one data set, backed by the dense matrix."""

    def __init__(self, A: np.ndarray, g: prism.Geometry):
        self.A = A
        self.sx, self.sy, self.nx, self.ny, self.nz = g.sx, g.sy, g.nx, g.ny, g.nz

    def matvec(self, x):
        return (self.A @ x.reshape(-1)).reshape(self.sx, self.sy)

    def rmatvec(self, v):
        return (self.A.T @ v.reshape(-1)).reshape(self.nz, self.nx, self.ny)
