"""Zero-padded FFT convolution and the error metric (sections 2 and 5).

Oracle (test infrastructure only).

u = crop( IFFT_M( K * FFT_M( pad(rho) ) ) ): rho is zero-padded from n to
M = 2n points per axis, transformed, multiplied by the real symbol K from
``kernel.half_spectrum``, transformed back (numpy normalisation: 1/M^3 on the
inverse) and cropped to the first n points per axis.  This is the plain,
unpruned form of the paper's size-8N transform pair.
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft


def solve(rho: np.ndarray, khalf: np.ndarray, workers: int | None = None) -> np.ndarray:
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape
    M = tuple(2 * v for v in n)
    if khalf.shape != (M[0], M[1], n[2] + 1):
        raise ValueError("symbol shape does not match the padded grid")
    workers = workers or os.cpu_count()
    F = scipy.fft.rfftn(rho, s=M, workers=workers)
    F *= khalf
    u = scipy.fft.irfftn(F, s=M, workers=workers)
    del F
    return np.ascontiguousarray(u[:n[0], :n[1], :n[2]])


def error_E(u: np.ndarray, u_ref: np.ndarray) -> float:
    """E = max|u - u_ref| / max|u_ref| over the grid (section 5)."""
    u = np.asarray(u, dtype=np.float64)
    u_ref = np.asarray(u_ref, dtype=np.float64)
    return float(np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref)))
