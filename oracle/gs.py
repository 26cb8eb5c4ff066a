"""Gaussian-sum approximation of U(r) = 1/(4 pi r) (section 2).

Oracle (test infrastructure only).

The paper approximates U by a sum of Gaussians obtained from sinc quadrature
of an integral representation.  Written out:

    1/r = (2/sqrt(pi)) * int_R exp(-r^2 e^{2t} + t) dt,

and the trapezoidal (sinc) rule with step hs at t_j = j*hs gives

    U(r) ~ sum_j w_j exp(-tau_j^2 r^2),  tau_j = e^{t_j},
    w_j = hs * tau_j / (2 pi^{3/2})          (the 1/(4 pi) included).

The budget eps is split into quarters eps' = eps/4 over three error sources:
* step: the integrand is analytic in the strip |Im t| < pi/4, so the
  discretisation error is about 2 exp(-pi^2/(2 hs)); hs = pi^2 / (2 ln(2/eps')).
* upper tail (t > t_max): relative error erfc(r e^{t_max}) <= eps' for r >= delta,
  so e^{t_max} = erfcinv(eps') / delta.
* lower tail (t < t_min): relative error <= (2/sqrt(pi)) r e^{t_min} <= eps'
  for r <= R, so e^{t_min} = eps' sqrt(pi) / (2 R).
The fit is then checked: max |U_GS/U - 1| over log-spaced r in [delta, R] must
not exceed eps; otherwise hs shrinks by 5 % and the fit is redone.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfcinv


def relative_error(tau, w, r):
    """|U_GS(r) / U(r) - 1| for an array of radii r."""
    out = np.empty_like(r)
    for s in range(0, r.size, 16384):
        rr = r[s:s + 16384]
        u = np.exp(-np.outer(rr * rr, tau * tau)) @ w
        out[s:s + 16384] = np.abs(4.0 * math.pi * rr * u - 1.0)
    return out


def gaussian_sum(eps: float, delta: float, R: float, n_check: int = 400_000,
                 max_shrink: int = 20):
    """Return (tau, w, max_rel_err) with max rel. error of U_GS on [delta, R] <= eps."""
    if not (0 < delta < R):
        raise ValueError("need 0 < delta < R")
    ep = eps / 4.0
    hs = math.pi ** 2 / (2.0 * math.log(2.0 / ep))
    t_max = math.log(float(erfcinv(ep)) / delta)
    t_min = math.log(ep * math.sqrt(math.pi) / (2.0 * R))
    r = np.exp(np.linspace(math.log(delta), math.log(R), n_check))
    for _ in range(max_shrink):
        j = np.arange(math.floor(t_min / hs), math.ceil(t_max / hs) + 1, dtype=np.float64)
        tau = np.exp(j * hs)
        w = hs * tau / (2.0 * math.pi ** 1.5)
        err = float(relative_error(tau, w, r).max())
        if err <= eps:
            return tau, w, err
        hs *= 0.95
    raise RuntimeError("Gaussian-sum fit did not reach the tolerance")
