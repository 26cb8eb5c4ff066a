"""FP64 CPU oracle for the free-space Poisson solve u = U * rho, U = 1/(4 pi |x|).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or run
anything in this package; only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the GPU library: it is an
independent, plain and slow restatement of the method of Exl (arXiv 1612.01799)
in numpy/scipy, written step by step from the paper:

* ``geometry``   grid, padded FFT period and the delta heuristic (sections 3-4)
* ``gs``         Gaussian-sum approximation of 1/(4 pi r) by sinc quadrature (section 2)
* ``modes``      1-D mode integrals of the truncated Gaussians, the factors of
                 the G-tensor (section 2), by adaptive Gauss-Kronrod as the paper does
* ``correction`` near-zone correction constants C0, C2 from the Taylor expansion (section 2)
* ``kernel``     kernel spectrum K = G-tensor + C0 - C2/6 |kappa|^2 (section 2)
* ``solve``      zero-padded FFT convolution and the error metric E (sections 2, 5)
* ``paper_form`` the correction by the paper's route: Laplacian from the
                 finite Fourier series of the density, an N-size FFT pair (sections 2-3)
* ``direct``     brute-force direct summation of the same discrete convolution
* ``analytic``   the paper's closed-form potentials for its test densities (section 5)

Every function is pinned by a ``-m "not gpu"`` test against values the paper
prints, closed forms, or brute force; see ``tests/test_oracle_*.py``.
"""
from .geometry import Geometry, geometry
from .gs import gaussian_sum
from .modes import mode_integrals
from .correction import correction
from .kernel import KernelSpectrum, kernel_spectrum, half_spectrum
from .solve import solve, error_E
from .paper_form import laplacian_fourier, solve_paper_form
from . import analytic, direct

__all__ = ["Geometry", "geometry", "gaussian_sum", "mode_integrals", "correction",
           "KernelSpectrum", "kernel_spectrum", "half_spectrum", "solve", "error_E",
           "laplacian_fourier", "solve_paper_form",
           "analytic", "direct"]
