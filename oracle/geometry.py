"""Grid geometry, padded period and the near-zone radius (sections 2-4).

Oracle (test infrastructure only).

Readings of the paper used here:
* The grid of each axis is ``linspace(a, b, n)`` (usage example, section 4):
  h = (b - a)/(n - 1), end points included.
* The zero padding doubles every axis, M = 2n, so the FFT period is P = M h and
  the kernel is truncated at T = P/2 = n h (section 2, the G-tensor with the
  padded transform).
* delta: the heuristic of section 3, min_q (b_q - a_q)/(50 n_q) floored at
  1e-3, is a length in the standardised frame (it must lie below the smallest
  standardised half-width); the physical radius is lambda times it, with
  lambda the largest half-width (section 2).
* R: the Gaussian sum must resolve 1/r over every distance between two grid
  points, i.e. up to the box diagonal sqrt(sum_q (b_q - a_q)^2) (twice the
  standardised box of section 2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Geometry:
    n: tuple
    a: tuple
    b: tuple
    h: tuple
    M: tuple
    P: tuple
    T: tuple
    lam: float
    delta: float
    R: float

    def kappa(self, q: int) -> np.ndarray:
        """Folded angular frequencies 2 pi k / P_q for k = 0..n_q."""
        k = np.arange(self.n[q] + 1, dtype=np.float64)
        return 2.0 * math.pi * k / self.P[q]


def geometry(box) -> Geometry:
    n = tuple(int(v) for v in box.n)
    a = tuple(float(v) for v in box.a)
    b = tuple(float(v) for v in box.b)
    h = tuple((b[q] - a[q]) / (n[q] - 1) for q in range(3))
    M = tuple(2 * n[q] for q in range(3))
    P = tuple(M[q] * h[q] for q in range(3))
    T = tuple(n[q] * h[q] for q in range(3))
    lam = max((b[q] - a[q]) / 2.0 for q in range(3))
    delta_std = max(1e-3, min((b[q] - a[q]) / (50.0 * n[q]) for q in range(3)))
    R = math.sqrt(sum((b[q] - a[q]) ** 2 for q in range(3)))
    return Geometry(n, a, b, h, M, P, T, lam, lam * delta_std, R)
