"""Brute-force direct summation of the discrete convolution.

Oracle (test infrastructure only).

The padded FFT convolution equals a circular convolution of the padded
density with the periodic kernel k = IFFT_M(K).  Because the density is zero
outside the first n points per axis and only the first n outputs are kept,
no wrap-around term reaches the output, so

    u[m] = sum_{j in [0,n)^3} k[(m - j) mod M] rho[j]

for m in [0, n)^3.  This O(n^6) sum checks padding, cropping and the
normalisation of ``solve`` without any FFT on the convolution path.
"""
from __future__ import annotations

import numpy as np
import scipy.fft


def periodic_kernel(khalf: np.ndarray, M) -> np.ndarray:
    return scipy.fft.irfftn(khalf, s=tuple(M))


def direct_solve(rho: np.ndarray, khalf: np.ndarray) -> np.ndarray:
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape
    M = tuple(2 * v for v in n)
    k = periodic_kernel(khalf, M)
    idx = [np.arange(v) for v in n]
    d = [(idx[q][:, None] - idx[q][None, :]) % M[q] for q in range(3)]   # (m_q, j_q)
    u = np.zeros(n)
    for m0 in range(n[0]):
        # kernel slab for this output plane: (j0, m1, j1, m2, j2)
        k0 = k[d[0][m0]]                                        # (j0, M1, M2)
        k01 = k0[:, d[1]]                                       # (j0, m1, j1, M2)
        k012 = k01[:, :, :, d[2]]                               # (j0, m1, j1, m2, j2)
        u[m0] = np.einsum("amben,abn->me", k012, rho)
    return u
