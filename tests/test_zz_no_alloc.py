"""The no-allocation batch entry point against psn_solve_batched, through the C ABI.

Two calls in a row, the second with a smaller input; each output must equal
the allocating entry point's output for the same inputs (same kernels, same
schedules: bitwise), and both must meet the oracle tolerances.  A batch whose
workspace exceeds the fixed scratch array is refused before any launch.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_common import TOL, max_rel, oracle_symbol, torch_cuda

pytestmark = pytest.mark.gpu
psn = pytest.importorskip("paper_1612_01799_amd")


def _entries(torch, spec):
    """spec: list of (n, L, dtype, seed) -> plans, device inputs, host inputs."""
    plans, rhos, host, cache = [], [], [], {}
    for n, L, dt, seed in spec:
        if (n, L, dt) not in cache:
            cache[(n, L, dt)] = psn.Plan(n, L, 1e-12, dt).build()
        plan = cache[(n, L, dt)]
        mix = W.draw_mixture(seed, 4, -L / 4, L / 4, 0.15 * L, 0.3 * L, 0.5, 1.5, W.Box.cube(L, n))
        r = W.mixture_density(mix)
        plans.append(plan)
        host.append(r)
        rhos.append(torch.from_numpy(r).to("cuda", plan.io_dtype()))
    return plans, rhos, host


def _check_call(torch, spec):
    plans, rhos, host = _entries(torch, spec)
    print("no-alloc batch: " + ", ".join(f"n={n} {dt}" for n, _, dt, _ in spec), flush=True)
    ref_out = psn.solve_batched(plans, rhos)
    outs = [torch.full_like(r, float("nan")) for r in rhos]
    psn.solve_batched_noalloc(plans, rhos, outs)
    torch.cuda.synchronize()
    for (n, L, dt, _), a, b, r in zip(spec, outs, ref_out, host):
        assert torch.equal(a, b), (n, dt)
        err = max_rel(a.double().cpu().numpy(), O.solve(r, oracle_symbol(n, L)))
        assert err <= TOL[dt], (n, dt, err)


def test_noalloc_batch_matches_allocating_batch():
    torch = torch_cuda()
    # first call: several sizes and precisions, about 70 MB of workspace
    _check_call(torch, [(96, 3.0, "f32", 1), (64, 2.5, "f32", 2), (48, 2.0, "split", 3), (64, 2.5, "f32", 4),
                        (32, 2.0, "f64", 5)])
    # second call, smaller: the array keeps the first call's contents, which
    # the passes must overwrite before reading
    _check_call(torch, [(32, 2.0, "f32", 6), (16, 1.5, "f64", 7)])


def test_noalloc_batch_refuses_oversize_workspace():
    torch = torch_cuda()
    plan = psn.Plan(160, 4.0, 1e-12, "f32").build()
    rhos = [torch.zeros((160,) * 3, device="cuda", dtype=torch.float32) for _ in range(3)]
    outs = [torch.full_like(r, 7.0) for r in rhos]
    with pytest.raises(psn.PsnError) as e:
        psn.solve_batched_noalloc([plan] * 3, rhos, outs)      # 3 x 98 MB > 256 MiB
    assert e.value.status == -7
    torch.cuda.synchronize()
    assert all(bool((o == 7.0).all()) for o in outs)           # nothing was enqueued
    psn.solve_batched_noalloc([plan] * 2, rhos[:2], outs[:2])  # 2 x 98 MB fits
    torch.cuda.synchronize()
    assert all(bool((o == 0).all()) for o in outs[:2])


def test_noalloc_batch_with_fourier_correction():
    """Plans that add the correction by the Fourier series keep its half
    spectrum in the workspace too: the same outputs as the allocating entry
    point, and the oracle's paper-form solve, on two calls in a row."""
    torch = torch_cuda()
    for n, L, seed in ((48, 2.5, 11), (24, 2.0, 12)):
        box = W.Box.cube(L, n)
        mix = W.draw_mixture(seed, 4, -L / 4, L / 4, 0.15 * L, 0.3 * L, 0.5, 1.5, box)
        r = W.mixture_density(mix)
        plans = [psn.Plan(n, L, 1e-12, "f32", correction="fourier").build(), psn.Plan(n, L, 1e-12, "f32").build()]
        rho = torch.from_numpy(r).to("cuda", torch.float32)
        print(f"no-alloc batch with the Fourier-series correction: n={n}", flush=True)
        ref_out = psn.solve_batched(plans, [rho, rho])
        outs = [torch.full_like(rho, float("nan")) for _ in plans]
        psn.solve_batched_noalloc(plans, [rho, rho], outs)
        torch.cuda.synchronize()
        for a, b in zip(outs, ref_out):
            assert torch.equal(a, b), n
        assert max_rel(outs[0].double().cpu().numpy(), O.solve_paper_form(r, box, 1e-12)) <= TOL["f32"]
        assert max_rel(outs[1].double().cpu().numpy(), O.solve(r, oracle_symbol(n, L))) <= TOL["f32"]
