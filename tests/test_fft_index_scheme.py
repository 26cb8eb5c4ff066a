"""The team FFT's index scheme, emulated in numpy for every compiled size.

The device transform (TeamFFT in csrc/psn_device.h) keeps E = n / T elements
per thread: slot e of thread t starts at input position t + T (e / R0) +
(e % R0) (n / R0), each stage runs E / R butterflies of radix R on
consecutive slots after multiplying by the stage twiddles, and the exchange
writes slot e to (b / Ns) Ns R + b % Ns + (e % R) Ns with b = t + T (e / R).
This test restates those formulas and the radix-plan rule, runs them on
random lines, and compares with numpy's FFT, so a wrong position, span or
twiddle step in the scheme fails here without a GPU.  The device code
itself is checked against the oracle by the GPU parity tests.
"""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def compiled_sizes():
    src = open(os.path.join(ROOT, "paper_1612_01799_amd", "csrc", "psn_internal.h")).read()
    m = re.search(r"#define PSN_FOR_EACH_SIZE\(X\)\s*\\\s*\n(.*)", src)
    return [int(v) for v in re.findall(r"X\((\d+)\)", m.group(1))]


def elems_per_thread(n, real_bytes):
    odd = n
    while odd % 2 == 0:
        odd //= 2
    cap = (8 if real_bytes == 8 else 16) if odd == 1 else 4
    oe = odd
    if oe > 15:
        oe = max(d for d in range(1, 10) if odd % d == 0)
        cap = 2
    return oe * min(n // odd, cap)


def make_plan(n, e):
    """Odd factors first, each merged with a factor 4 or 2 where both what is
    left of n and E allow it; then the largest power of two up to 16 that
    divides what is left and the power-of-two part of E."""
    plan, rem = [], n
    for f in (5, 3):
        while rem % f == 0:
            r = next((f * p for p in (4, 2, 1) if rem % (f * p) == 0 and e % (f * p) == 0), None)
            if r is None:
                return None
            plan.append(r)
            rem //= r
    e2 = e & -e
    while rem > 1:
        r = 16
        while r > 1 and (rem % r or e2 % r):
            r //= 2
        if r == 1:
            return None
        plan.append(r)
        rem //= r
    return plan


def team_fft(x, n, t_count, sign, rev):
    """One line through the team scheme: returns the output and the plan."""
    e_count = n // t_count
    plan = make_plan(n, e_count)
    assert plan is not None and all(e_count % r == 0 for r in plan)
    if rev:
        plan = plan[::-1]
    tw = np.exp(-2j * np.pi * np.arange(2 * n) / (2 * n))
    r0 = plan[0]
    d = np.array([[x[t + t_count * (e // r0) + (e % r0) * (n // r0)] for e in range(e_count)]
                  for t in range(t_count)])
    lds = np.zeros(n, complex)
    ns = 1
    for i, r in enumerate(plan):
        if i > 0:
            d = np.array([[lds[t + t_count * (e // r) + (e % r) * (n // r)] for e in range(e_count)]
                          for t in range(t_count)])
        step = 2 * n // (ns * r)
        m = np.arange(r)
        dft = np.exp(sign * 2j * np.pi * np.outer(m, m) / r)
        for t in range(t_count):
            for s in range(e_count // r):
                v = d[t, s * r:(s + 1) * r]
                if ns > 1:
                    w = tw[m * ((t + t_count * s) % ns) * step]
                    v = v * (w if sign < 0 else np.conj(w))
                d[t, s * r:(s + 1) * r] = dft @ v
        if i + 1 < len(plan):
            lds[:] = np.nan
            for t in range(t_count):
                for e in range(e_count):
                    b = t + t_count * (e // r)
                    lds[(b // ns) * ns * r + b % ns + (e % r) * ns] = d[t, e]
            assert not np.isnan(lds).any(), "exchange leaves a hole"
        ns *= r
    rl = plan[-1]
    out = np.full(n, np.nan, complex)
    for t in range(t_count):
        for e in range(e_count):
            out[t + t_count * (e // rl) + (e % rl) * (n // rl)] = d[t, e]
    return out, plan


def _cases():
    seen = set()
    for n in compiled_sizes():
        es = {elems_per_thread(n, 4), elems_per_thread(n, 8)}
        odd = n // (n & -n)
        if odd > 1:
            es.add(2 * odd)  # the half-length candidate of the axis-1 passes
        for e in sorted(es):
            if n % e == 0 and (n, e) not in seen:
                seen.add((n, e))
                yield n, e
        if n >= 16 and odd == 1:
            # the half-length chains of the middle pass on the paired layout
            h = n // 2
            for e in (min(8, h), min(4, h)):
                if (h, e) not in seen:
                    seen.add((h, e))
                    yield h, e


@pytest.mark.parametrize("n,e", list(_cases()))
def test_team_transform_matches_numpy(n, e):
    rng = np.random.default_rng(n * 100 + e)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for sign in (-1, 1):
        ref = np.fft.fft(x) if sign < 0 else np.fft.ifft(x) * n
        for rev in (False, True):
            y, _ = team_fft(x, n, n // e, sign, rev)
            assert np.max(np.abs(y - ref)) <= 1e-10 * n * np.max(np.abs(x))


def test_forward_output_order_is_reverse_plan_input_order():
    """A forward pass and an inverse with the radices reversed meet in the same
    register layout, which the middle pass relies on to multiply by K in place."""
    for n, e in _cases():
        t_count = n // e
        plan = make_plan(n, e)
        rl_fwd, r0_rev = plan[-1], plan[::-1][0]
        assert rl_fwd == r0_rev
        for t in (0, t_count - 1):
            for k in range(e):
                fwd_out = t + t_count * (k // rl_fwd) + (k % rl_fwd) * (n // rl_fwd)
                rev_in = t + t_count * (k // r0_rev) + (k % r0_rev) * (n // r0_rev)
                assert fwd_out == rev_in


@pytest.mark.parametrize("n,e,plan", [(160, 20, [20, 4, 2]), (96, 12, [12, 4, 2]), (320, 20, [20, 4, 4]),
                                      (384, 12, [12, 4, 4, 2]), (12, 12, [12]), (160, 10, [10, 2, 2, 2, 2]),
                                      (512, 8, [8, 8, 8]), (512, 16, [16, 16, 2]), (256, 16, [16, 16]),
                                      (162, 18, [6, 3, 3, 3])])
def test_plans_merge_odd_factors(n, e, plan):
    assert make_plan(n, e) == plan


@pytest.mark.parametrize("r1,r2", [(4, 5), (4, 3), (2, 5), (2, 3)])
def test_prime_factor_index_maps(r1, r2):
    """Good-Thomas: input n = (r2 n1 + r1 n2) mod R and output
    k = (r2 t1 k1 + r1 t2 k2) mod R with t1 r2 = 1 (mod r1), t2 r1 = 1 (mod r2)
    turn a length-R DFT into r2 DFTs of length r1 then r1 of length r2, with
    no twiddles between them."""
    r = r1 * r2
    t1 = next(v for v in range(1, r1 + 1) if (r2 * v) % r1 == 1 % r1)
    t2 = next(v for v in range(1, r2) if (r1 * v) % r2 == 1)
    rng = np.random.default_rng(r)
    x = rng.standard_normal(r) + 1j * rng.standard_normal(r)
    for sign in (-1, 1):
        a = np.array([[x[(r2 * n1 + r1 * n2) % r] for n1 in range(r1)] for n2 in range(r2)])
        a = np.array([np.exp(sign * 2j * np.pi * np.outer(np.arange(r1), np.arange(r1)) / r1) @ row for row in a])
        out = np.zeros(r, complex)
        w2 = np.exp(sign * 2j * np.pi * np.outer(np.arange(r2), np.arange(r2)) / r2)
        for k1 in range(r1):
            b = w2 @ a[:, k1]
            for k2 in range(r2):
                out[(r2 * t1 * k1 + r1 * t2 * k2) % r] = b[k2]
        ref = np.fft.fft(x) if sign < 0 else np.fft.ifft(x) * r
        assert np.max(np.abs(out - ref)) <= 1e-12 * r


@pytest.mark.parametrize("n", [16, 64, 512])
def test_paired_middle_pass_split(n):
    """The middle pass on the paired layout: a line x of n samples split by
    decimation in time into four half-length chains (even and odd samples,
    with and without the pre-twiddle w^j), joined by a radix-2 combine,
    multiplied by the folded kernel through its sum and difference over the
    two joined outputs, split again by decimation in frequency into four
    half-length inverses, and recombined with w^-j.  The result must equal
    the plain zero-padded length-2n convolution cropped to n samples (both
    unnormalised)."""
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    kfold = rng.standard_normal(n + 1)                     # K at folded index 0..n
    k = np.arange(2 * n)
    kfull = kfold[np.minimum(k, 2 * n - k)]
    ref = (np.fft.ifft(kfull * np.fft.fft(x, 2 * n)) * 2 * n)[:n]

    h = n // 2
    w = np.exp(-2j * np.pi * np.arange(2 * n) / (2 * n))   # w^j, j < 2n
    i = np.arange(h)
    xe, xo = x[0::2], x[1::2]
    A, B = np.fft.fft(xe), np.fft.fft(xo)
    C, D = np.fft.fft(xe * w[2 * i]), np.fft.fft(xo * w[2 * i + 1])
    m = np.arange(h)
    W = w[2 * m]                                           # exp(-2 pi i m / n)
    out = []
    for a, b, odd in ((A, B, 0), (C, D, 1)):
        k0, k1 = kfold[2 * m + odd], kfold[n - 2 * m - odd]
        ks, kd = k0 + k1, k0 - k1
        p = ks * a + kd * (W * b)
        q = ks * b + kd * (np.conj(W) * a)
        out.append((np.fft.ifft(p) * h, np.fft.ifft(q) * h))
    (P, Q), (R, S) = out
    u = np.empty(n, complex)
    u[0::2] = P + np.conj(w[2 * i]) * R
    u[1::2] = Q + np.conj(w[2 * i + 1]) * S
    assert np.max(np.abs(u - ref)) <= 1e-12 * n * np.max(np.abs(ref))


def test_paired_w2_index_is_a_permutation():
    """The paired W2 layout maps every (i0, k1, k2) to its own element, keeps
    each slot row of a tile (B columns x an i0 pair) contiguous, and puts the
    two i0 of a column next to each other."""
    n, bl = 16, 8
    kb, m = 4, 2 * n                      # the k1 block of n = 16
    blk = n * n * kb + 512

    def slot(k1):
        return 0 if k1 == 0 else 1 if k1 == n else (2 * k1 if k1 < n else 2 * (m - k1) + 1)

    def at(i0, k1, k2):
        sl = slot(k1)
        return (sl // kb) * blk + ((i0 >> 1) * (n // bl) + k2 // bl) * (2 * kb * bl) + (sl % kb) * 2 * bl \
            + (k2 % bl) * 2 + (i0 & 1)

    idx = [at(i0, k1, k2) for i0 in range(n) for k1 in range(m) for k2 in range(n)]
    assert len(set(idx)) == len(idx)
    assert at(4, 3, 9) + 1 == at(5, 3, 9)
    row = sorted(at(i0, 3, k2) for i0 in (6, 7) for k2 in range(8, 16))
    assert row == list(range(row[0], row[0] + 16))
