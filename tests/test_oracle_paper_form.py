"""The paper-form correction of the oracle (Laplacian by an N-size FFT pair),
pinned without reference to its own code:

* the Laplacian of a resolved periodic test function against its closed form;
* the printed errors E of Tables 1, 3, 5 and 7 (cube boxes), which the paper
  computed with this very form, to their printed digits;
* agreement with the folded form (the correction symbol added to the padded
  spectrum) to far below the method's error for a resolved density, and a
  clear disagreement when the correction's sign or the Fourier period is
  wrong (so the comparison can see such slips).
"""
import math

import numpy as np
import pytest

import oracle as O
import paper_cases as PC
import workloads as W

G = PC.load()


def test_laplacian_of_trig_polynomial():
    """cos(2 pi a x / P0) sin(2 pi b y / P1) cos(2 pi c z / P2) on the periodic
    grid x_i = a0 + i h: the Laplacian is -(2 pi)^2 (a^2/P0^2 + b^2/P1^2 + c^2/P2^2) times it."""
    n, h = (12, 10, 8), (0.3, 0.2, 0.5)
    P = [n[q] * h[q] for q in range(3)]
    x = [np.arange(n[q]) * h[q] - 1.0 for q in range(3)]
    a, b, c = 2, 3, 1
    f = (np.cos(2 * np.pi * a * x[0] / P[0])[:, None, None] * np.sin(2 * np.pi * b * x[1] / P[1])[None, :, None]
         * np.cos(2 * np.pi * c * x[2] / P[2])[None, None, :])
    lap = O.laplacian_fourier(f, h)
    ref = -(2 * np.pi) ** 2 * (a ** 2 / P[0] ** 2 + b ** 2 / P[1] ** 2 + c ** 2 / P[2] ** 2) * f
    assert np.max(np.abs(lap - ref)) <= 1e-12 * np.max(np.abs(ref))


def _cube_entries():
    out = []
    for e in G["digits"] + G["three_digits"]:
        if e["table"] in (1, 3, 5, 7) and e["n"] <= 32:
            out.append(e)
    return out


@pytest.mark.parametrize("entry", _cube_entries(), ids=[PC.name(e) for e in _cube_entries()])
def test_paper_form_reproduces_printed_error(entry):
    box, rho, ustar = PC.case(entry)
    E = O.error_E(O.solve_paper_form(rho, box, entry.get("eps", 1e-12)), ustar)
    digits = 4 if entry in G["digits"] else 3
    half = 0.5 * 10 ** (math.floor(math.log10(entry["E"])) - (digits - 1)) * 1.0001
    assert abs(E - entry["E"]) <= half, (E, entry["E"])


def test_paper_form_agrees_with_fold_for_resolved_density():
    mix = W.config_single()                 # sigma = 1 Gaussian, n = 32 on [-6, 6]^3
    rho = W.mixture_density(mix)
    u_fold = O.solve(rho, O.half_spectrum(O.kernel_spectrum(mix.box, 1e-12)))
    u_paper = O.solve_paper_form(rho, mix.box, 1e-12)
    scale = np.max(np.abs(u_fold))
    assert np.max(np.abs(u_paper - u_fold)) <= 1e-13 * scale
    # the comparison sees a wrong sign of the Laplacian term, or the padded period
    ks = O.kernel_spectrum(mix.box, 1e-12, with_correction=False)
    C0, C2 = O.correction(ks.tau, ks.w, ks.geom.delta)
    I1 = O.solve(rho, O.half_spectrum(ks))
    wrong_sign = I1 + C0 * rho - (C2 / 6) * O.laplacian_fourier(rho, ks.geom.h)
    wrong_period = I1 + C0 * rho + (C2 / 6) * O.laplacian_fourier(rho, [2 * v for v in ks.geom.h])
    assert np.max(np.abs(wrong_sign - u_fold)) > 1e3 * np.max(np.abs(u_paper - u_fold))
    assert np.max(np.abs(wrong_period - u_fold)) > 1e3 * np.max(np.abs(u_paper - u_fold))
