"""1-D mode integrals: the factors of the G-tensor (section 2).

Oracle (test infrastructure only).

For one Gaussian exp(-tau^2 y^2) truncated to [-T, T] and a folded frequency
kappa = 2 pi k / P, the paper's G-tensor factor is the cosine transform

    a(tau, kappa) = 2 * int_0^T exp(-tau^2 y^2) cos(kappa y) dy,

computed, as the paper does, by one-dimensional adaptive Gauss-Kronrod
quadrature.  Two regimes have an exact reduction that quadrature need not
resolve and that are used as they stand:

* tau*T >= 6.1: the tail beyond T is below exp(-37) relative, so
  a = sqrt(pi)/tau * exp(-kappa^2 / (4 tau^2))  (the Gaussian's Fourier transform);
* tau*T < 1:   a = 2 int_0^T cos(kappa y) dy + 2 int_0^T expm1(-tau^2 y^2) cos(kappa y) dy,
  where the first term is exactly 2T for k = 0 and 0 otherwise (kappa T = pi k);
  the smooth remainder is integrated by composite Gauss-Legendre.

Everything in between goes to adaptive Gauss-Kronrod (GK21, scipy's
``quad_vec``).  The alternative closed form through the Faddeeva function is
provided only as a cross-check for the tests.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad_vec
from scipy.special import erf, wofz

BIG = 6.1
SMALL = 1.0


def _gl_nodes(T: float, panels: int, order: int = 16):
    x, wt = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(0.0, T, panels + 1)
    half = 0.5 * np.diff(edges)
    mid = 0.5 * (edges[1:] + edges[:-1])
    y = (mid[:, None] + half[:, None] * x[None, :]).ravel()
    wy = (half[:, None] * wt[None, :]).ravel()
    return y, wy


def mode_integrals(tau, T: float, kappa, gk_tol: float = 1e-15):
    """Matrix a[j, k] = 2 int_0^T exp(-tau_j^2 y^2) cos(kappa_k y) dy."""
    tau = np.asarray(tau, dtype=np.float64)
    kappa = np.asarray(kappa, dtype=np.float64)
    A = np.empty((tau.size, kappa.size))
    tT = tau * T
    big = tT >= BIG
    small = tT < SMALL
    mid = ~(big | small)

    if big.any():
        tb = tau[big][:, None]
        A[big] = math.sqrt(math.pi) / tb * np.exp(-(kappa[None, :] ** 2) / (4.0 * tb * tb))

    if small.any():
        kmax = int(round(kappa[-1] * T / math.pi))
        y, wy = _gl_nodes(T, kmax // 2 + 8)
        ts = tau[small]
        E = np.expm1(-np.outer(ts * ts, y * y)) * wy[None, :]
        A[small] = 2.0 * (E @ np.cos(np.outer(y, kappa)))
        A[small, 0] += 2.0 * T

    for j in np.nonzero(mid)[0]:
        t = tau[j]
        a0 = math.sqrt(math.pi) * math.erf(t * T) / t
        f = lambda y, t=t: 2.0 * math.exp(-t * t * y * y) * np.cos(kappa * y)
        val, _err = quad_vec(f, 0.0, T, epsabs=gk_tol * a0, epsrel=0.0, norm="max",
                             quadrature="gk21", limit=200000)
        A[j] = val
    return A


def mode_integrals_gk(tau, T: float, kappa, gk_tol: float = 1e-15):
    """Adaptive Gauss-Kronrod for every term (slow; cross-check only)."""
    kappa = np.asarray(kappa, dtype=np.float64)
    A = np.empty((len(tau), kappa.size))
    for j, t in enumerate(np.asarray(tau, dtype=np.float64)):
        a0 = math.sqrt(math.pi) * math.erf(t * T) / t
        f = lambda y, t=t: 2.0 * math.exp(-t * t * y * y) * np.cos(kappa * y)
        A[j], _ = quad_vec(f, 0.0, T, epsabs=gk_tol * a0, epsrel=0.0, norm="max",
                           quadrature="gk21", limit=200000)
    return A


def mode_integrals_faddeeva(tau, T: float, kappa):
    """Closed form sqrt(pi)/tau Re[exp(-kappa^2/4tau^2) - exp(-tau^2 T^2 + i kappa T) w(kappa/2tau + i tau T)].

    Cross-check only: it loses digits when tau*T << 1.
    """
    tau = np.asarray(tau, dtype=np.float64)[:, None]
    kappa = np.asarray(kappa, dtype=np.float64)[None, :]
    z = kappa / (2.0 * tau) + 1j * tau * T
    val = np.exp(-kappa ** 2 / (4.0 * tau ** 2)) - np.exp(-(tau * T) ** 2 + 1j * kappa * T) * wofz(z)
    return math.sqrt(math.pi) / tau * val.real


def mode_at_zero(tau, T: float):
    """Exact a(tau, 0) = sqrt(pi) erf(tau T) / tau."""
    tau = np.asarray(tau, dtype=np.float64)
    return math.sqrt(math.pi) * erf(tau * T) / tau
