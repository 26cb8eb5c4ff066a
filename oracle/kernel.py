"""Kernel spectrum: G-tensor plus folded near-zone correction (section 2).

Oracle (test infrastructure only).

The smooth part I_1 is a convolution with the truncated Gaussian sum; its
Fourier symbol on the padded grid is the G-tensor

    G[k0, k1, k2] = sum_j w_j a_j^(0)(k0) a_j^(1)(k1) a_j^(2)(k2),

with a_j^(q) the 1-D mode integrals of axis q.  The correction C0 rho +
(C2/6) Laplace(rho) has the symbol C0 - (C2/6) |kappa|^2, which is added to the
same spectrum so one padded convolution returns I_1 + I_delta.  The symbol is
real and even in every axis, so only the octant k_q = 0..n_q is formed; the
folded index min(k, M - k) recovers any frequency.  No h^3 factor and no 1/M^3
normalisation appear: the inverse FFT carries 1/M^3 (numpy convention).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .correction import correction
from .geometry import Geometry, geometry
from .gs import gaussian_sum
from .modes import mode_integrals


@dataclass
class KernelSpectrum:
    geom: Geometry
    eps: float
    tau: np.ndarray
    w: np.ndarray
    gs_err: float
    C0: float
    C2: float
    octant: np.ndarray            # (n0+1, n1+1, n2+1), FP64

    @property
    def S(self) -> int:
        """Index of the last Gaussian-sum term (terms j = 0..S)."""
        return self.tau.size - 1


def kernel_spectrum(box, eps: float = 1e-12, with_correction: bool = True) -> KernelSpectrum:
    g = geometry(box)
    tau, w, err = gaussian_sum(eps, g.delta, g.R)
    if with_correction:
        C0, C2 = correction(tau, w, g.delta)
    else:
        C0, C2 = 0.0, 0.0
    cache = {}
    A = []
    for q in range(3):
        key = (g.T[q], g.n[q])
        if key not in cache:
            cache[key] = mode_integrals(tau, g.T[q], g.kappa(q))
        A.append(cache[key])
    n0, n1, n2 = (v + 1 for v in g.n)
    B = (w[:, None, None] * A[0][:, :, None] * A[1][:, None, :]).reshape(tau.size, n0 * n1)
    K = (B.T @ A[2]).reshape(n0, n1, n2)
    k2 = [g.kappa(q) ** 2 for q in range(3)]
    K += C0 - (C2 / 6.0) * (k2[0][:, None, None] + k2[1][None, :, None] + k2[2][None, None, :])
    return KernelSpectrum(g, eps, tau, w, err, C0, C2, K)


def fold(M: int) -> np.ndarray:
    k = np.arange(M)
    return np.minimum(k, M - k)


def half_spectrum(ks: KernelSpectrum) -> np.ndarray:
    """Full-length symbol on the rfftn half grid: shape (M0, M1, n2 + 1)."""
    g = ks.geom
    f0, f1 = fold(g.M[0]), fold(g.M[1])
    return np.ascontiguousarray(ks.octant[f0][:, f1, :])
