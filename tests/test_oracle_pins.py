"""Oracle vs the errors E printed in the paper's Tables 1-7 (section 5).

The paper's E compares its FP64 solution with the closed-form potential, so
reproducing the printed digits pins the whole oracle (grid, padding period,
truncation T, normalisation, Gaussian sum and correction) at once.
"""
import math

import pytest

import oracle as O
import paper_cases as PC

G = PC.load()
_cache = {}


def _symbol(box, eps):
    key = (box.a, box.b, box.n, eps)
    if key not in _cache:
        _cache[key] = O.half_spectrum(O.kernel_spectrum(box, eps))
    return _cache[key]


def _E(entry):
    box, rho, ustar = PC.case(entry)
    return O.error_E(O.solve(rho, _symbol(box, entry.get("eps", 1e-12))), ustar)


def _half_unit(E, digits):
    return 0.5 * 10 ** (math.floor(math.log10(E)) - (digits - 1)) * 1.0001


@pytest.mark.parametrize("entry", G["digits"], ids=[PC.name(e) for e in G["digits"]])
def test_printed_error_four_digits(entry):
    E = _E(entry)
    assert abs(E - entry["E"]) <= _half_unit(entry["E"], 4), (E, entry["E"])


@pytest.mark.parametrize("entry", G["three_digits"], ids=[PC.name(e) for e in G["three_digits"]])
def test_printed_error_three_digits(entry):
    E = _E(entry)
    assert abs(E - entry["E"]) <= _half_unit(entry["E"], 3), (E, entry["E"])


@pytest.mark.parametrize("entry", G["bounds"], ids=[PC.name(e) for e in G["bounds"]])
def test_converged_rows(entry):
    assert _E(entry) <= entry["max"]


def test_without_correction_error_is_about_1e6():
    """Section 3: without I_delta the method's error is of order max(delta^2, eps) ~ 1e-6."""
    box, rho, ustar = PC.case(G["bounds"][0])
    ks = O.kernel_spectrum(box, 1e-12, with_correction=False)
    E = O.error_E(O.solve(rho, O.half_spectrum(ks)), ustar)
    assert 1e-7 < E < 1e-5
