"""Brute-force discrete Fourier transforms (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The FFT2 of Sec. 2.7.1 is the plain 2-D DFT; this module writes its definition out
as a matrix product with explicitly built DFT matrices, O(N^2) per axis, so that
an FFT kernel of any radix can be checked against the definition itself.
Convention: forward X[k] = sum_n x[n] exp(-2 pi i n k / N), inverse unscaled with
the opposite sign.  Pins: tests/test_oracle_bttb.py checks these against numpy.fft
and Parseval's identity.
"""
from __future__ import annotations

import numpy as np


def dft_matrix(N: int, sign: int = -1) -> np.ndarray:
    n = np.arange(N)
    # reduce n*k mod N in integers before scaling, so the angle is exact for large N
    e = np.outer(n, n) % N
    return np.exp(sign * 2j * np.pi * e / N)


def dft(x: np.ndarray, axis: int = -1, sign: int = -1) -> np.ndarray:
    x = np.asarray(x, dtype=np.complex128)
    F = dft_matrix(x.shape[axis], sign)
    return np.moveaxis(np.tensordot(np.moveaxis(x, axis, -1), F, axes=([-1], [0])), -1, axis)


def dft2(x: np.ndarray, sign: int = -1) -> np.ndarray:
    return dft(dft(x, axis=-1, sign=sign), axis=-2, sign=sign)
