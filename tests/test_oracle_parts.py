"""Oracle building blocks against closed forms, independent quadrature and brute force."""
import math

import mpmath
import numpy as np
import pytest
from scipy.integrate import quad

import oracle as O
import workloads as W
import importlib
OC = importlib.import_module("oracle.correction")
from oracle import gs as OG
from oracle import modes as OM


# ------------------------------------------------------------------ geometry
def test_geometry_cube_readings():
    g = O.geometry(W.Box.cube(6.0, 32))
    assert g.h[0] == pytest.approx(12 / 31, rel=1e-15)
    assert g.M == (64, 64, 64)
    assert g.T[0] == pytest.approx(32 * 12 / 31, rel=1e-15)
    assert g.P[0] == pytest.approx(2 * g.T[0], rel=1e-15)
    assert g.delta == pytest.approx(6 * 12 / (50 * 32), rel=1e-15)        # 0.045
    assert g.R == pytest.approx(12 * math.sqrt(3), rel=1e-15)
    assert O.geometry(W.Box.cube(12.0, 512)).delta == pytest.approx(0.012, rel=1e-12)
    assert O.geometry(W.Box.cube(2.0, 64)).delta == pytest.approx(2 * 1e-3 * 1.25, rel=1e-12)


def test_delta_floor():
    g = O.geometry(W.Box.cube(1.0, 1000))
    assert g.delta == pytest.approx(1e-3, rel=1e-15)


@pytest.mark.parametrize("a,b,n", [((-300.0,) * 3, (300.0,) * 3, (16,) * 3),
                                   ((-1.0, -7.0, -2.0), (3.0, 5.0, 2.5), (16, 96, 24)),
                                   ((-40.0, -10.0, -10.0), (40.0, 10.0, 10.0), (8, 16, 16)),
                                   ((-12.0,) * 3, (12.0,) * 3, (512,) * 3)])
def test_delta_lies_in_the_papers_interval(a, b, n):
    """Section 2 asks for delta in (0, min_q (b_q - a_q) / (2 lambda)) in the
    standardised frame x = lambda x' + c, and section 3 says its heuristic
    lies there whenever lambda <= 25 min_q n_q.  So the near-zone ball, of
    physical radius lambda * delta, lies inside the box's shortest half-edge.
    A reading that scaled the heuristic by lambda once more leaves the
    interval on the first and third boxes (0.75 -> 225 against 1, and
    0.025 -> 1 against 0.25)."""
    box = W.Box(a, b, n)
    g = O.geometry(box)
    lam = max(0.5 * (b[q] - a[q]) for q in range(3))
    assert lam <= 25 * min(n)
    d_std = g.delta / lam
    assert 1e-3 <= d_std < min((b[q] - a[q]) / (2 * lam) for q in range(3))
    assert g.delta < min(0.5 * (b[q] - a[q]) for q in range(3))


# ------------------------------------------------------------------ Gaussian sum
@pytest.mark.parametrize("L,n,eps", [(6.0, 32, 1e-12), (8.0, 128, 1e-12), (12.0, 512, 1e-12),
                                     (2.0, 16, 1e-8), (10.0, 256, 1e-14)])
def test_gaussian_sum_relative_error(L, n, eps):
    g = O.geometry(W.Box.cube(L, n))
    tau, w, err = O.gaussian_sum(eps, g.delta, g.R)
    assert err <= eps
    # independent sample: random radii, not the fit's own check grid
    rng = np.random.default_rng(7)
    r = np.exp(rng.uniform(math.log(g.delta), math.log(g.R), 20000))
    assert OG.relative_error(tau, w, r).max() <= eps
    assert np.all(np.diff(tau) > 0) and np.all(w > 0)


def test_gaussian_sum_term_count():
    for L, n in [(6.0, 32), (8.0, 128), (10.0, 256), (12.0, 512)]:
        g = O.geometry(W.Box.cube(L, n))
        tau, _, _ = O.gaussian_sum(1e-12, g.delta, g.R)
        assert 220 <= tau.size <= 240


def test_gaussian_sum_mpmath_point():
    g = O.geometry(W.Box.cube(6.0, 32))
    tau, w, _ = O.gaussian_sum(1e-12, g.delta, g.R)
    for r in (g.delta, 0.3, 1.7, g.R):
        s = mpmath.fsum(mpmath.mpf(float(wj)) * mpmath.exp(-(mpmath.mpf(float(tj)) * r) ** 2)
                        for tj, wj in zip(tau, w))
        assert abs(float(s * 4 * mpmath.pi * r) - 1.0) <= 1e-12


# ------------------------------------------------------------------ mode integrals
def _modes_setup(L=2.0, n=16, eps=1e-12):
    g = O.geometry(W.Box.cube(L, n))
    tau, w, _ = O.gaussian_sum(eps, g.delta, g.R)
    return g, tau, w


def test_mode_zero_frequency_closed_form():
    g, tau, _ = _modes_setup()
    A = O.mode_integrals(tau, g.T[0], g.kappa(0))
    ref = OM.mode_at_zero(tau, g.T[0])
    assert np.max(np.abs(A[:, 0] - ref) / ref) <= 1e-14


def test_modes_branches_vs_full_gauss_kronrod():
    g, tau, _ = _modes_setup()
    A = O.mode_integrals(tau, g.T[0], g.kappa(0))
    B = OM.mode_integrals_gk(tau, g.T[0], g.kappa(0))
    a0 = OM.mode_at_zero(tau, g.T[0])
    assert np.max(np.abs(A - B) / a0[:, None]) <= 2e-15


def test_modes_vs_faddeeva_closed_form():
    g, tau, _ = _modes_setup(6.0, 32)
    A = O.mode_integrals(tau, g.T[0], g.kappa(0))
    F = OM.mode_integrals_faddeeva(tau, g.T[0], g.kappa(0))
    a0 = OM.mode_at_zero(tau, g.T[0])
    big = tau * g.T[0] >= 1.0
    assert np.max(np.abs(A[big] - F[big]) / a0[big, None]) <= 1e-14


@pytest.mark.parametrize("tT,k", [(0.05, 0), (0.05, 7), (0.8, 3), (2.0, 1), (2.0, 16), (5.0, 9),
                                  (7.0, 2)])
def test_modes_mpmath(tT, k):
    T = 1.3
    n = 16
    tau = tT / T
    kappa = math.pi * k / T                      # kappa T = pi k
    mpmath.mp.dps = 30
    f = lambda y: 2 * mpmath.exp(-(tau * y) ** 2) * mpmath.cos(kappa * y)
    ref = float(mpmath.quad(f, mpmath.linspace(0, T, 2 * k + 3)))
    got = O.mode_integrals(np.array([tau]), T, math.pi * np.arange(n + 1) / T)[0, k]
    assert abs(got - ref) <= 1e-15 * float(OM.mode_at_zero(np.array([tau]), T)[0])


# ------------------------------------------------------------------ correction
@pytest.mark.parametrize("L,n", [(2.0, 16), (6.0, 32), (12.0, 512)])
def test_correction_vs_quadrature(L, n):
    g = O.geometry(W.Box.cube(L, n))
    tau, w, _ = O.gaussian_sum(1e-12, g.delta, g.R)
    C0, C2 = O.correction(tau, w, g.delta)
    ugs = lambda r: float(np.dot(w, np.exp(-(tau * r) ** 2)))
    q0, _ = quad(lambda r: r - 4 * math.pi * r * r * ugs(r), 0, g.delta, epsabs=0, epsrel=1e-13, limit=200)
    q2, _ = quad(lambda r: r ** 3 - 4 * math.pi * r ** 4 * ugs(r), 0, g.delta, epsabs=0, epsrel=1e-13, limit=200)
    assert C0 == pytest.approx(q0, rel=1e-10)
    assert C2 == pytest.approx(q2, rel=1e-10)


def test_radial_moments_series_and_closed_form_meet():
    d = 0.02
    tau = np.array([0.5 / d * (1 - 1e-9), 0.5 / d * (1 + 1e-9)])
    i2, i4 = OC.radial_moments(tau, d)
    assert i2[0] == pytest.approx(i2[1], rel=1e-8)
    assert i4[0] == pytest.approx(i4[1], rel=1e-8)
    mpmath.mp.dps = 40
    for t in (3.0, 25.0, 400.0):
        r2 = float(mpmath.quad(lambda r: r ** 2 * mpmath.exp(-(t * r) ** 2), [0, d]))
        r4 = float(mpmath.quad(lambda r: r ** 4 * mpmath.exp(-(t * r) ** 2), [0, d]))
        a, b = OC.radial_moments(np.array([t]), d)
        assert a[0] == pytest.approx(r2, rel=1e-13)
        assert b[0] == pytest.approx(r4, rel=1e-13)


# ------------------------------------------------------------------ kernel spectrum
@pytest.mark.parametrize("L,n", [(6.0, 32), (2.0, 24)])
def test_kernel_at_zero_is_cube_integral(L, n):
    """K(0) = int over [-T,T]^3 of 1/(4 pi |y|) = T^2 (3 ln(2+sqrt 3) - pi/2) / pi."""
    ks = O.kernel_spectrum(W.Box.cube(L, n), 1e-12)
    T = ks.geom.T[0]
    exact = T * T * (3 * math.log(2 + math.sqrt(3)) - math.pi / 2) / math.pi
    assert ks.octant[0, 0, 0] == pytest.approx(exact, rel=5e-12)


def test_kernel_symmetry_and_fold():
    ks = O.kernel_spectrum(W.Box.cube(2.0, 12), 1e-12)
    K = ks.octant
    assert np.allclose(K, K.transpose(1, 0, 2), rtol=0, atol=1e-15 * abs(K).max())
    assert np.allclose(K, K.transpose(2, 1, 0), rtol=0, atol=1e-15 * abs(K).max())
    H = O.half_spectrum(ks)
    M = ks.geom.M[0]
    for k in range(1, M):
        assert np.array_equal(H[k], H[M - k])
        assert np.array_equal(H[:, k], H[:, M - k])


# ------------------------------------------------------------------ convolution
@pytest.mark.parametrize("n", [(8, 8, 8), (6, 8, 10)])
def test_fft_solve_equals_direct_sum(n):
    box = W.Box((-1.0, -1.2, -0.9), (1.0, 1.1, 1.3), n)
    rng = np.random.default_rng(3)
    rho = rng.standard_normal(n)
    H = O.half_spectrum(O.kernel_spectrum(box, 1e-10))
    u = O.solve(rho, H)
    v = O.direct.direct_solve(rho, H)
    assert np.max(np.abs(u - v)) <= 1e-13 * np.max(np.abs(v))
