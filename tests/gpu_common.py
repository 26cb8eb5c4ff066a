"""Shared helpers for GPU parity tests (oracle results are cached per case)."""
import functools

import numpy as np
import pytest

import oracle as O
import workloads as W

TOL = {"f64": 1e-12, "split": 1e-10, "f32": 1e-5}   # max-norm relative error vs the FP64 oracle


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    return torch


@functools.lru_cache(maxsize=None)
def oracle_symbol(n, L, tol=1e-12):
    return O.half_spectrum(O.kernel_spectrum(W.Box.cube(L, n), tol))


@functools.lru_cache(maxsize=None)
def oracle_octant(n, L, tol=1e-12):
    return O.kernel_spectrum(W.Box.cube(L, n), tol).octant


def gpu_solve(psn, torch, n, L, dtype, rho_np, tol=1e-12, plan=None):
    plan = plan or psn.Plan(n, L, tol, dtype).build()
    rho = torch.from_numpy(np.ascontiguousarray(rho_np)).to("cuda", plan.io_dtype())
    u = plan.solve(rho)
    torch.cuda.synchronize()
    return u.double().cpu().numpy()


def max_rel(u, ref):
    return float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))
