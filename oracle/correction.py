"""Near-zone correction constants (section 2).

Oracle (test infrastructure only).

Inside the ball B_delta the Gaussian sum is replaced by the exact kernel: the
correction I_delta(x) = int_{B_delta} (U - U_GS)(y) rho(x - y) dy is evaluated
with the third-order Taylor polynomial of rho around x.  Odd orders and the
off-diagonal Hessian entries integrate to zero against a radial function, and
int y_q^2 f = (1/3) int |y|^2 f, so

    I_delta ~ C0 * rho(x) + (C2 / 6) * Laplace(rho)(x),
    C0 = int_{B_delta} (U - U_GS) dy,   C2 = int_{B_delta} |y|^2 (U - U_GS) dy.

In spherical coordinates, with I2(tau) = int_0^delta r^2 e^{-tau^2 r^2} dr and
I4(tau) = int_0^delta r^4 e^{-tau^2 r^2} dr:

    C0 = delta^2/2 - 4 pi sum_j w_j I2(tau_j),
    C2 = delta^4/4 - 4 pi sum_j w_j I4(tau_j).

I2 and I4 use their erf closed forms, or their Taylor series when tau*delta <
0.5, where the closed forms cancel.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def _series(tau, delta, p, terms=40):
    # int_0^delta r^p exp(-tau^2 r^2) dr = sum_m (-tau^2)^m delta^(2m+p+1) / (m! (2m+p+1))
    x = -(tau * tau) * delta * delta
    out = np.zeros_like(tau)
    term = np.ones_like(tau)          # x^m / m!
    for m in range(terms):
        out += term / (2 * m + p + 1)
        term = term * x / (m + 1)
    return out * delta ** (p + 1)


def radial_moments(tau, delta):
    """Return (I2(tau), I4(tau)) for an array of tau."""
    tau = np.asarray(tau, dtype=np.float64)
    x = tau * delta
    e = np.exp(-x * x)
    sp = math.sqrt(math.pi)
    with np.errstate(divide="ignore", invalid="ignore"):
        i2 = sp * erf(x) / (4 * tau ** 3) - delta * e / (2 * tau ** 2)
        i4 = 3 * sp * erf(x) / (8 * tau ** 5) - e * (3 * delta / (4 * tau ** 4) + delta ** 3 / (2 * tau ** 2))
    sm = x < 0.5
    if sm.any():
        i2 = np.where(sm, _series(tau, delta, 2), i2)
        i4 = np.where(sm, _series(tau, delta, 4), i4)
    return i2, i4


def correction(tau, w, delta: float):
    """Return (C0, C2)."""
    i2, i4 = radial_moments(tau, delta)
    w = np.asarray(w, dtype=np.float64)
    C0 = delta ** 2 / 2.0 - 4.0 * math.pi * float(np.dot(w, i2))
    C2 = delta ** 4 / 4.0 - 4.0 * math.pi * float(np.dot(w, i4))
    return C0, C2
