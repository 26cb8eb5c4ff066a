"""The near-zone correction by the paper's route (psn_plan_set_correction with
PSN_CORRECTION_FOURIER: Laplacian from the density's size-N Fourier series)
against the oracle's paper-form solve, element by element."""
import math

import numpy as np
import pytest

import oracle as O
import paper_cases as PC
import workloads as W
from gpu_common import TOL, max_rel, torch_cuda

pytestmark = pytest.mark.gpu
psn = pytest.importorskip("paper_1612_01799_amd")


def _mix(n, L, seed):
    return W.mixture_density(W.draw_mixture(seed, 5, -L / 3, L / 3, 0.25 * L / 2, 0.45 * L / 2, 0.5, 1.5,
                                            W.Box.cube(L, n)))


def _solve(torch, plan, rho_np, inplace=False):
    rho = torch.from_numpy(np.ascontiguousarray(rho_np)).to("cuda", plan.io_dtype())
    u = plan.solve(rho, out=rho if inplace else None)
    torch.cuda.synchronize()
    return u.double().cpu().numpy()


@pytest.mark.parametrize("n", [8, 12, 16, 24, 48, 64, 96, 128, 160, 162])
@pytest.mark.parametrize("dtype", ["f64", "f32", "split"])
def test_fourier_correction_matches_oracle(n, dtype):
    torch = torch_cuda()
    L = 2.0 + n / 64.0
    box = W.Box.cube(L, n)
    rho = _mix(n, L, 700 + n)
    ref = O.solve_paper_form(rho, box, 1e-12)
    plan = psn.Plan(n, L, 1e-12, dtype, correction="fourier").build()
    assert plan.info()["correction"] == psn.CORRECTION_FOURIER
    err = max_rel(_solve(torch, plan, rho), ref)
    print(f"fourier correction n={n} {dtype}: {err:.3e}", flush=True)
    assert err <= TOL[dtype]


def test_fourier_correction_kernel_is_the_g_tensor():
    """With the Fourier-series correction the spectrum holds the G-tensor alone."""
    torch_cuda()
    n, L = 32, 2.5
    plan = psn.Plan(n, L, 1e-12, "f64", correction="fourier").build()
    ks = O.kernel_spectrum(W.Box.cube(L, n), 1e-12, with_correction=False)
    assert np.max(np.abs(plan.kernel_octant() - ks.octant)) <= 1e-13 * abs(ks.octant[0, 0, 0])


def test_fourier_correction_in_place_and_box():
    torch = torch_cuda()
    box = W.Box((-3.0, -2.0, -1.0), (2.0, 3.5, 5.0), (32, 32, 32))
    rho = W.mixture_density(W.draw_mixture(41, 4, -0.3, 0.6, 0.35, 0.6, 0.5, 1.5, box))
    ref = O.solve_paper_form(rho, box, 1e-12)
    plan = psn.Plan(32, box=(box.a, box.b), tol=1e-12, dtype="f64", correction="fourier").build()
    assert max_rel(_solve(torch, plan, rho, inplace=True), ref) <= TOL["f64"]


def _entries():
    g = PC.load()
    return [e for e in g["digits"] + g["three_digits"] if e["table"] in (1, 3, 5, 7)]


@pytest.mark.parametrize("entry", _entries(), ids=[PC.name(e) for e in _entries()])
def test_paper_tables_fourier_correction_fp64(entry):
    """Tables 1, 3, 5 and 7 were computed with this form of the correction."""
    torch = torch_cuda()
    box, rho, ustar = PC.case(entry)
    plan = psn.Plan(box.n[0], box=(box.a, box.b), tol=entry.get("eps", 1e-12), dtype="f64",
                    correction="fourier").build()
    E = O.error_E(_solve(torch, plan, rho), ustar)
    digits = 4 if entry in PC.load()["digits"] else 3
    assert abs(E - entry["E"]) <= 0.5 * 10 ** (math.floor(math.log10(entry["E"])) - (digits - 1)) * 1.0001


def test_batch_mixes_correction_modes():
    """Entries of one size with either form of the correction share launches."""
    torch = torch_cuda()
    n, L = 48, 2.5
    box = W.Box.cube(L, n)
    pf = psn.Plan(n, L, 1e-12, "f64", correction="fourier").build()
    pd = psn.Plan(n, L, 1e-12, "f64").build()
    rhos_np = [_mix(n, L, 800 + i) for i in range(4)]
    rhos = [torch.from_numpy(r).to("cuda") for r in rhos_np]
    plans = [pf, pd, pf, pd]
    outs = psn.solve_batched(plans, rhos)
    outs2 = [torch.empty_like(r) for r in rhos]
    psn.solve_batched_noalloc(plans, rhos, outs2)
    torch.cuda.synchronize()
    sym = O.half_spectrum(O.kernel_spectrum(box, 1e-12))
    for p, r, u, u2 in zip(plans, rhos_np, outs, outs2):
        ref = O.solve_paper_form(r, box, 1e-12) if p is pf else O.solve(r, sym)
        assert max_rel(u.cpu().numpy(), ref) <= TOL["f64"]
        assert torch.equal(u, u2)


def test_correction_mode_fixed_after_build():
    torch_cuda()
    p = psn.Plan(16, 1.0, 1e-12, "f64").build()
    assert psn._lib.psn_plan_set_correction(p.handle, psn.CORRECTION_FOURIER) == -5
