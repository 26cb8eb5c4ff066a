"""The near-zone correction by the paper's own route (section 2, last paragraph; section 3).

Oracle (test infrastructure only).

The correction I_delta ~ C0 rho + (C2/6) Laplace(rho) (Taylor expansion of
the density in the delta-ball, see ``correction``) is not folded into the
padded spectrum here.  The Laplacian is taken from the finite Fourier series
of the density on its own grid, where differentiation is a scalar
multiplication: one forward and one backward FFT of size N = n0 n1 n2
(section 3).  The smooth part I_1 is the zero-padded convolution with the
G-tensor alone, and

    u = I_1 + C0 rho + (C2 / 6) Laplace_N(rho).

Reading: the finite Fourier series of the n_q samples of an axis is their
discrete Fourier transform, period n_q h_q, frequencies kappa = 2 pi k / (n_q h_q)
with k the signed index (-n_q/2 .. n_q/2 - 1); the Laplacian's symbol
-sum_q kappa_q^2 is even, so the Nyquist term needs no further choice.
"""
from __future__ import annotations

import math

import numpy as np

from .correction import correction
from .kernel import half_spectrum, kernel_spectrum
from .solve import solve


def laplacian_fourier(rho: np.ndarray, h) -> np.ndarray:
    """Laplace(rho) from the finite Fourier series of the samples (period n_q h_q per axis)."""
    rho = np.asarray(rho, dtype=np.float64)
    sym = np.zeros(rho.shape)
    for q in range(3):
        kap = 2.0 * math.pi * np.fft.fftfreq(rho.shape[q], d=h[q])
        shape = [1, 1, 1]
        shape[q] = -1
        sym = sym - (kap ** 2).reshape(shape)
    return np.real(np.fft.ifftn(np.fft.fftn(rho) * sym))


def solve_paper_form(rho: np.ndarray, box, eps: float = 1e-12, workers: int | None = None) -> np.ndarray:
    """u = I_1 (padded convolution with the G-tensor only) + C0 rho + (C2/6) Laplace_N(rho)."""
    ks = kernel_spectrum(box, eps, with_correction=False)
    C0, C2 = correction(ks.tau, ks.w, ks.geom.delta)
    rho = np.asarray(rho, dtype=np.float64)
    u = solve(rho, half_spectrum(ks), workers=workers)
    return u + C0 * rho + (C2 / 6.0) * laplacian_fourier(rho, ks.geom.h)
