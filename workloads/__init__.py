"""Seeded synthetic inputs for the free-space Poisson solve.

This module only *generates densities*: grids, the paper's analytic test
densities rho (section 5) and the seeded Gaussian-mixture workloads.  It holds
none of the solver's arithmetic (no Gaussian-sum, no mode integrals, no FFT),
so both the FP64 CPU oracle and the GPU path may draw their inputs from it.

Conventions
-----------
* Grids follow the paper's usage example: each axis is ``linspace(a, b, n)``
  with both end points included, so ``h = (b - a) / (n - 1)`` (section 4).
* Arrays are C-order ``[i0][i1][i2]`` (``i2`` contiguous), FP64.
* A seeded draw uses ``numpy.random.default_rng(seed)`` in the fixed order
  centres (k x 3), widths (k), signs (k), magnitudes (k).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "axis", "Box", "Mixture", "mixture_density", "draw_mixture",
    "paper_gaussian", "paper_two_gaussians", "paper_bump",
    "paper_anisotropic", "paper_oscillating",
    "config_single", "config_n128", "config_n256", "config_n512",
    "config_batched", "BATCH_EDGES",
]


def axis(a: float, b: float, n: int) -> np.ndarray:
    """Grid points of one axis: ``a + i*(b-a)/(n-1)``, end points included."""
    if n < 2:
        raise ValueError("an axis needs at least two points")
    i = np.arange(n, dtype=np.float64)
    return a + i * ((b - a) / (n - 1))


@dataclass(frozen=True)
class Box:
    """Rectangular box [a_q, b_q] with n_q points per axis (q = 0, 1, 2)."""
    a: tuple
    b: tuple
    n: tuple

    @staticmethod
    def cube(L: float, n: int) -> "Box":
        return Box((-L, -L, -L), (L, L, L), (n, n, n))

    def axes(self):
        return [axis(self.a[q], self.b[q], self.n[q]) for q in range(3)]

    def centre(self):
        return tuple(0.5 * (self.a[q] + self.b[q]) for q in range(3))


@dataclass
class Mixture:
    """Sum of normalised isotropic Gaussians q_g * pi^-3/2 s_g^-3 exp(-|x-c_g|^2/s_g^2)."""
    centres: np.ndarray        # (k, 3)
    sigmas: np.ndarray         # (k,)
    charges: np.ndarray        # (k,)
    box: Box = field(default=None)


def mixture_density(mix: Mixture, box: Box | None = None) -> np.ndarray:
    """FP64 density of a Gaussian mixture sampled on ``box``.

    Each term is separable, so the sum is formed as a matrix product of
    per-axis factors (exact up to rounding; no approximation).
    """
    box = box or mix.box
    x0, x1, x2 = box.axes()
    k = len(mix.sigmas)
    s = np.asarray(mix.sigmas, dtype=np.float64)
    c = np.asarray(mix.centres, dtype=np.float64).reshape(k, 3)
    coef = np.asarray(mix.charges, dtype=np.float64) * math.pi ** -1.5 / s ** 3
    g0 = np.exp(-((x0[None, :] - c[:, 0:1]) ** 2) / s[:, None] ** 2) * coef[:, None]
    g1 = np.exp(-((x1[None, :] - c[:, 1:2]) ** 2) / s[:, None] ** 2)
    g2 = np.exp(-((x2[None, :] - c[:, 2:3]) ** 2) / s[:, None] ** 2)
    a01 = (g0[:, :, None] * g1[:, None, :]).reshape(k, -1)      # (k, n0*n1)
    rho = a01.T @ g2                                            # (n0*n1, n2)
    return np.ascontiguousarray(rho.reshape(box.n[0], box.n[1], box.n[2]))


def draw_mixture(seed: int, k: int, centre_lo: float, centre_hi: float,
                 sigma_lo: float, sigma_hi: float, q_lo: float, q_hi: float,
                 box: Box) -> Mixture:
    """Seeded mixture draw: centres, widths, signs, magnitudes (that order).

    If the total charge is below 1e-3 in magnitude the last charge's sign is
    flipped, so every drawn mixture has a nonzero monopole.
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(centre_lo, centre_hi, size=(k, 3))
    sigmas = rng.uniform(sigma_lo, sigma_hi, size=k)
    signs = np.where(rng.integers(0, 2, size=k) == 0, -1.0, 1.0)
    mags = rng.uniform(q_lo, q_hi, size=k)
    q = signs * mags
    if abs(q.sum()) < 1e-3:
        q[-1] = -q[-1]
    return Mixture(centres, sigmas, q, box)


# ---------------------------------------------------------------------------
# Benchmark workloads (seeded Gaussian mixtures)
# ---------------------------------------------------------------------------

def config_single() -> Mixture:
    """n = 32 on [-6, 6]^3: one normalised Gaussian, sigma = 1, at the origin."""
    box = Box.cube(6.0, 32)
    return Mixture(np.zeros((1, 3)), np.array([1.0]), np.array([1.0]), box)


def config_n128(seed: int = 1002) -> Mixture:
    """n = 128 on [-8, 8]^3: 8 Gaussians, centres U[-2,2]^3, sigma U[0.5,1.2], q = +-U[0.5,1.5]."""
    return draw_mixture(seed, 8, -2.0, 2.0, 0.5, 1.2, 0.5, 1.5, Box.cube(8.0, 128))


def config_n256(seed: int = 1003) -> Mixture:
    """n = 256 on [-10, 10]^3: 32 Gaussians, centres U[-4,4]^3, sigma U[0.4,1.5], q = +-1."""
    return draw_mixture(seed, 32, -4.0, 4.0, 0.4, 1.5, 1.0, 1.0, Box.cube(10.0, 256))


def config_n512(seed: int = 1005) -> Mixture:
    """n = 512 on [-12, 12]^3: 128 Gaussians, centres U[-6,6]^3, sigma U[0.3,2.0], q = +-1."""
    return draw_mixture(seed, 128, -6.0, 6.0, 0.3, 2.0, 1.0, 1.0, Box.cube(12.0, 512))


BATCH_EDGES = (48, 64, 96, 128, 160)


def config_batched(seed: int = 1004, count: int = 64, edges=BATCH_EDGES):
    """Mixed-size batch: edges drawn from ``edges``, spacing h = 0.1.

    Problem p has ``n_p`` points per axis on [-L_p, L_p]^3 with
    L_p = 0.05 (n_p - 1), and 4 Gaussians with centres U[-L_p/4, L_p/4]^3,
    sigma U[0.3, 1.0] and charges +-U[0.5, 1.5].  Each problem's mixture uses
    its own sub-seed ``seed * 1000 + p``.
    """
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(edges), size=count)
    out = []
    for p, n in enumerate(ns):
        n = int(n)
        L = 0.05 * (n - 1)
        out.append(draw_mixture(seed * 1000 + p, 4, -L / 4, L / 4, 0.3, 1.0, 0.5, 1.5,
                                Box.cube(L, n)))
    return out


# ---------------------------------------------------------------------------
# The paper's analytic test densities (section 5).  Each is -Laplace(u*) of a
# closed-form potential u*; the potentials live with the oracle.
# ---------------------------------------------------------------------------

def _r2(box: Box, c):
    x0, x1, x2 = box.axes()
    return ((x0 - c[0])[:, None, None] ** 2 + (x1 - c[1])[None, :, None] ** 2
            + (x2 - c[2])[None, None, :] ** 2)


def paper_gaussian(box: Box, sigma: float, c=None) -> np.ndarray:
    """Gaussian of section 5.1: (2 pi)^-3/2 sigma^-3 exp(-|x-c|^2 / (2 sigma^2)), c = box centre."""
    c = box.centre() if c is None else c
    return (2 * math.pi) ** -1.5 / sigma ** 3 * np.exp(-_r2(box, c) / (2 * sigma ** 2))


def paper_two_gaussians(box: Box, d, s1: float, s2: float, c=None) -> np.ndarray:
    """Superposition of section 5.2: half the sum of Gaussians at c+d (width s1) and c-d (width s2)."""
    c = box.centre() if c is None else c
    cp = tuple(c[q] + d[q] for q in range(3))
    cm = tuple(c[q] - d[q] for q in range(3))
    return 0.5 * (paper_gaussian(box, s1, cp) + paper_gaussian(box, s2, cm))


def paper_bump(box: Box, d: float, R: float, c=None) -> np.ndarray:
    """Bump of section 5.3, as -Laplace of u* = exp(-d / (1 - r^2/R^2)) for r < R.

    The printed formula is garbled; this is the density whose potential is the
    printed u* (exponent -d R^2/(R^2 - r^2), polynomial term -2 d R^2 r^2).
    """
    c = box.centre() if c is None else c
    r2 = _r2(box, c)
    inside = r2 < R * R
    out = np.zeros_like(r2)
    q = r2[inside]
    den = R * R - q
    out[inside] = (2 * d * R * R * (3 * R ** 4 - 2 * R * R * q - q * q - 2 * d * R * R * q)
                   / den ** 4 * np.exp(-d * R * R / den))
    return out


def paper_anisotropic(box: Box, sig, c=None) -> np.ndarray:
    """Anisotropic density of section 5.4: -Laplace of exp(-sum_q (x_q-c_q)^2 / s_q^2)."""
    c = box.centre() if c is None else c
    x = box.axes()
    e = [np.exp(-((x[q] - c[q]) ** 2) / sig[q] ** 2) for q in range(3)]
    p = [4 * (x[q] - c[q]) ** 2 / sig[q] ** 4 - 2 / sig[q] ** 2 for q in range(3)]
    g = e[0][:, None, None] * e[1][None, :, None] * e[2][None, None, :]
    s = p[0][:, None, None] + p[1][None, :, None] + p[2][None, None, :]
    return -s * g


def paper_oscillating(box: Box, sigma: float, omega: float, c=None) -> np.ndarray:
    """Oscillating density of section 5.5, as -Laplace of exp(-r^2/s^2) cos(w r^2).

    The printed formula has a sign slip; this is the density whose potential is
    the printed u* (the 4 w^2 r^2 cos term enters with a plus sign).
    """
    c = box.centre() if c is None else c
    r2 = _r2(box, c)
    E = np.exp(-r2 / sigma ** 2)
    cw = np.cos(omega * r2)
    sw = np.sin(omega * r2)
    return (E * (6 * omega * sw + 4 * omega ** 2 * r2 * cw)
            - (4 * r2 / sigma ** 4 - 6 / sigma ** 2) * E * cw
            - 8 * omega * r2 / sigma ** 2 * E * sw)
