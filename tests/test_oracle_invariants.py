"""Oracle solve: closed-form potentials of the workloads and invariants of U * rho."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W


def test_single_gaussian_closed_form():
    """n = 32 on [-6,6]^3, sigma = 1: potential erf(|x|)/(4 pi |x|)."""
    mix = W.config_single()
    rho = W.mixture_density(mix)
    H = O.half_spectrum(O.kernel_spectrum(mix.box, 1e-12))
    E = O.error_E(O.solve(rho, H), O.analytic.mixture(mix))
    assert E <= 1e-10


def test_mixture_n128_closed_form():
    """n = 128 on [-8,8]^3, 8 Gaussians: tails at the box edge are ~1e-11 of the peak."""
    mix = W.config_n128()
    rho = W.mixture_density(mix)
    H = O.half_spectrum(O.kernel_spectrum(mix.box, 1e-12))
    E = O.error_E(O.solve(rho, H), O.analytic.mixture(mix))
    assert E <= 1e-10


@pytest.fixture(scope="module")
def small():
    box = W.Box.cube(3.0, 24)
    H = O.half_spectrum(O.kernel_spectrum(box, 1e-12))
    return box, H


def _mix(box, seed, k=3):
    return W.draw_mixture(seed, k, -0.8, 0.8, 0.35, 0.6, 0.5, 1.5, box)


def test_linearity(small):
    box, H = small
    r1 = W.mixture_density(_mix(box, 1))
    r2 = W.mixture_density(_mix(box, 2))
    lhs = O.solve(2.5 * r1 - 0.75 * r2, H)
    rhs = 2.5 * O.solve(r1, H) - 0.75 * O.solve(r2, H)
    assert np.max(np.abs(lhs - rhs)) <= 1e-14 * np.max(np.abs(lhs))


def test_axis_permutation(small):
    box, H = small
    rho = W.mixture_density(_mix(box, 3))
    u = O.solve(rho, H)
    for perm in [(1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)]:
        v = O.solve(np.ascontiguousarray(rho.transpose(perm)), H)
        assert np.max(np.abs(v - u.transpose(perm))) <= 1e-14 * np.max(np.abs(u))


def test_self_adjoint(small):
    box, H = small
    r1 = W.mixture_density(_mix(box, 4))
    r2 = W.mixture_density(_mix(box, 5))
    a = float(np.sum(r2 * O.solve(r1, H)))
    b = float(np.sum(r1 * O.solve(r2, H)))
    assert a == pytest.approx(b, rel=1e-13)


def test_translation_by_one_cell(small):
    box, H = small
    rng = np.random.default_rng(9)
    rho = np.zeros(box.n)
    rho[6:14, 7:15, 5:13] = rng.standard_normal((8, 8, 8))
    u = O.solve(rho, H)
    v = O.solve(np.roll(rho, (1, 2, 3), axis=(0, 1, 2)), H)
    ref = np.roll(u, (1, 2, 3), axis=(0, 1, 2))
    assert np.max(np.abs(v[1:, 2:, 3:] - ref[1:, 2:, 3:])) <= 1e-13 * np.max(np.abs(u))


def test_positive_density_gives_positive_potential(small):
    box, H = small
    mix = W.draw_mixture(11, 3, -0.8, 0.8, 0.4, 0.6, 0.5, 1.5, box)
    mix.charges[:] = np.abs(mix.charges)
    u = O.solve(W.mixture_density(mix), H)
    assert np.all(u > 0)


def test_far_field_monopole():
    """Far from compact charges the potential is sum_i q_i / (4 pi |x - c_i|)."""
    box = W.Box.cube(6.0, 64)
    H = O.half_spectrum(O.kernel_spectrum(box, 1e-12))
    mix = W.Mixture(np.array([[0.3, -0.2, 0.1], [-0.4, 0.5, 0.0]]), np.array([0.6, 0.7]),
                    np.array([1.0, -0.6]), box)
    u = O.solve(W.mixture_density(mix), H)
    x = box.axes()
    X0, X1, X2 = np.meshgrid(*x, indexing="ij")
    far = np.ones(box.n, bool)
    ref = np.zeros(box.n)
    for c, s, q in zip(mix.centres, mix.sigmas, mix.charges):
        d = np.sqrt((X0 - c[0]) ** 2 + (X1 - c[1]) ** 2 + (X2 - c[2]) ** 2)
        far &= d >= 6 * s
        ref += q / (4 * math.pi * np.maximum(d, 1e-30))
    assert far.sum() > 1000
    assert np.max(np.abs(u[far] - ref[far])) <= 1e-10 * np.max(np.abs(ref[far]))
