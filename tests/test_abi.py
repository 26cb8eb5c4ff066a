"""C ABI on the host: the library loads, exports every declared symbol, and its
host-only work (argument checks, geometry, Gaussian-sum table) matches the
oracle.  No device work is done here."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psn.h")

psn = pytest.importorskip("paper_1612_01799_amd")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psn_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ["psn_plan_create", "psn_kernel_build", "psn_solve", "psn_solve_batched", "psn_plan_query",
              "psn_plan_destroy", "psn_strerror"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(psn.library_path())
    for s in declared_symbols():
        assert hasattr(lib, s), s


@pytest.mark.parametrize("n,ok", [(8, True), (12, True), (16, True), (24, True), (48, True), (96, True),
                                  (160, True), (162, True), (512, True), (7, False), (14, False), (2, False), (0, False),
                                  (-8, False), (42, False), (1024 * 8, False)])
def test_size_rules(n, ok):
    assert psn.size_supported(n) == ok
    if not ok:
        with pytest.raises(psn.PsnError) as e:
            psn.Plan(n, 1.0)
        assert e.value.status == -2


@pytest.mark.parametrize("L,tol,dt", [(0.0, 1e-12, "f32"), (-1.0, 1e-12, "f32"), (float("inf"), 1e-12, "f32"),
                                      (float("nan"), 1e-12, "f32"), (1.0, 1e-16, "f32"), (1.0, 1e-3, "f32"),
                                      (1.0, float("nan"), "f64")])
def test_invalid_arguments(L, tol, dt):
    with pytest.raises(psn.PsnError) as e:
        psn.Plan(16, L, tol, dt)
    assert e.value.status == -1


def test_bad_dtype_and_null_out():
    lib = psn._lib
    h = ctypes.c_void_p()
    assert lib.psn_plan_create(16, 1.0, 1e-12, 7, ctypes.byref(h)) == -1
    assert lib.psn_plan_create(16, 1.0, 1e-12, 0, None) == -1
    assert lib.psn_plan_query(None, None) == -1
    lib.psn_plan_destroy(None)


@pytest.mark.parametrize("n,L,tol", [(32, 6.0, 1e-12), (128, 8.0, 1e-12), (16, 2.0, 1e-14), (48, 2.35, 1e-8)])
def test_geometry_and_gaussian_sum_match_oracle(n, L, tol):
    p = psn.Plan(n, L, tol, "f64")
    info = p.info()
    g = O.geometry(W.Box.cube(L, n))
    assert info["h"] == pytest.approx(g.h[0], rel=1e-15)
    assert info["T"] == pytest.approx(g.T[0], rel=1e-15)
    assert info["period"] == pytest.approx(g.P[0], rel=1e-15)
    assert info["delta"] == pytest.approx(g.delta, rel=1e-15)
    assert info["R"] == pytest.approx(g.R, rel=1e-15)
    assert info["built"] == 0 and info["device_bytes"] == 0
    assert info["eps_achieved"] <= tol
    tau_o, w_o, _ = O.gaussian_sum(tol, g.delta, g.R)
    tau, w = p.gs_table()
    assert info["terms"] == tau.size == tau_o.size
    assert np.max(np.abs(tau / tau_o - 1)) <= 1e-14
    assert np.max(np.abs(w / w_o - 1)) <= 1e-14


@pytest.mark.parametrize("a,b,n", [((-3, -2, -1), (2, 3.5, 5), 32), ((-3, -2, -2), (1, 3, 4), 16),
                                   ((-2, -4, -6), (2, 4, 6), 64)])
def test_box_geometry_matches_oracle(a, b, n):
    p = psn.Plan(n, box=(a, b), tol=1e-12, dtype="f64")
    info = p.info()
    g = O.geometry(W.Box(a, b, (n, n, n)))
    for q in range(3):
        assert info["h3"][q] == pytest.approx(g.h[q], rel=1e-15)
        assert info["T3"][q] == pytest.approx(g.T[q], rel=1e-15)
        assert info["a"][q] == a[q] and info["b"][q] == b[q]
    assert info["delta"] == pytest.approx(g.delta, rel=1e-15)
    assert info["R"] == pytest.approx(g.R, rel=1e-15)
    assert info["L"] == pytest.approx(g.lam, rel=1e-15)
    tau_o, _, _ = O.gaussian_sum(1e-12, g.delta, g.R)
    assert info["terms"] == tau_o.size


def test_box_rejects_empty_axes():
    with pytest.raises(psn.PsnError) as e:
        psn.Plan(16, box=((0, 0, 0), (1, 0, 1)))
    assert e.value.status == -1
    with pytest.raises(psn.PsnError) as e:
        psn.Plan(16, box=((0, 0, 0), (1, float("nan"), 1)))
    assert e.value.status == -1


def test_solve_before_build_is_a_state_error():
    p = psn.Plan(16, 1.0, 1e-12, "f32")
    lib = psn._lib
    buf = ctypes.create_string_buffer(16 * 16 * 16 * 4)
    assert lib.psn_solve(p.handle, ctypes.cast(buf, ctypes.c_void_p), ctypes.cast(buf, ctypes.c_void_p), None) == -5
    assert lib.psn_solve(p.handle, None, ctypes.cast(buf, ctypes.c_void_p), None) == -1
    k = np.empty(17 ** 3)
    assert lib.psn_kernel_download(p.handle, k.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == -5
    P = ctypes.c_void_p
    arr = (P * 1)(p.handle)
    bufs = (P * 1)(ctypes.cast(buf, P))
    assert lib.psn_solve_batched(1, arr, bufs, bufs, None) == -5
    assert lib.psn_solve_batched(0, None, None, None, None) == 0
    assert lib.psn_solve_batched(-1, None, None, None, None) == -1
    assert lib.psn_solve_batched(1, None, None, None, None) == -1


def test_algorithmic_bytes():
    n = 512
    # W1: n^3 complex, written and read twice; W2: 2 n^3 complex, accessed four
    # times; split precision stores W1 in 12 bytes and W2 in FP64
    for dt, (bio, b1, b2, bk) in {"f32": (4, 8, 8, 4), "f64": (8, 16, 16, 8), "split": (8, 12, 16, 8)}.items():
        info = psn.Plan(n, 12.0, 1e-12, dt).info()
        assert info["algorithmic_bytes"] == 2 * bio * n ** 3 + 4 * b1 * n ** 3 + 8 * b2 * n ** 3 + bk * (n + 1) ** 3


def test_schedule_override_validation():
    p = psn.Plan(32, 1.0, 1e-12, "f32")
    p.set_schedule(2, 1)
    assert p.info()["schedule"] == (2, 1) and p.info()["tuned"] == 0
    for bad in [(-1, 0), (4, 0), (0, 4)]:
        with pytest.raises(psn.PsnError) as e:
            p.set_schedule(*bad)
        assert e.value.status == -1


def test_strerror():
    for st in range(-7, 1):
        assert psn._lib.psn_strerror(st)
    assert psn._lib.psn_strerror(-99) == b"unknown status"


def test_binding_rejects_host_tensors():
    """A host tensor never reaches the kernels as a device pointer."""
    import torch
    p = psn.Plan(16, 1.0, 1e-12, "f32")
    rho = torch.zeros((16, 16, 16), dtype=torch.float32)
    with pytest.raises(ValueError):
        p.solve(rho)
    with pytest.raises(ValueError):
        psn.solve_batched([p], [rho])
    with pytest.raises(ValueError):
        psn.solve_batched([p, p], [rho])


def test_noalloc_batch_host_checks():
    """Argument and state errors of the no-allocation batch are found on the
    host before any device work."""
    lib = psn._lib
    p = psn.Plan(16, 1.0, 1e-12, "f32")
    buf = ctypes.create_string_buffer(16 * 16 * 16 * 4)
    P = ctypes.c_void_p
    arr = (P * 1)(p.handle)
    bufs = (P * 1)(ctypes.cast(buf, P))
    assert lib.psn_solve_batched_noalloc(1, arr, bufs, bufs, None) == -5
    assert lib.psn_solve_batched_noalloc(0, None, None, None, None) == 0
    assert lib.psn_solve_batched_noalloc(-1, None, None, None, None) == -1
    assert lib.psn_solve_batched_noalloc(1, None, None, None, None) == -1


def test_correction_option_host_checks():
    p = psn.Plan(16, 1.0, 1e-12, "f64")
    assert p.info()["correction"] == psn.CORRECTION_FOLDED
    lib = psn._lib
    assert lib.psn_plan_set_correction(p.handle, 7) == -1
    assert lib.psn_plan_set_correction(None, 0) == -1
    assert lib.psn_plan_set_correction(p.handle, psn.CORRECTION_FOURIER) == 0
    assert p.info()["correction"] == psn.CORRECTION_FOURIER
    q = psn.Plan(16, 1.0, 1e-12, "f32", correction="fourier")
    assert q.info()["correction"] == psn.CORRECTION_FOURIER


def test_grid_plan_host_checks():
    lib = psn._lib
    P = ctypes.c_void_p
    h = P()
    a = (ctypes.c_double * 3)(-1, -1, -1)
    b = (ctypes.c_double * 3)(1, 2, 3)
    for bad, st in (((16, 24, 14), -2), ((16, 0, 32), -2), ((7, 16, 16), -2)):
        nn = (ctypes.c_int * 3)(*bad)
        assert lib.psn_plan_create_grid(nn, a, b, 1e-12, 1, ctypes.byref(h)) == st
    assert lib.psn_plan_create_grid(None, a, b, 1e-12, 1, ctypes.byref(h)) == -1
    p = psn.Plan((16, 24, 32), box=((-1, -1, -1), (1, 2, 3)), tol=1e-12, dtype="f64")
    info = p.info()
    assert info["n3"] == (16, 24, 32)
    g = O.geometry(W.Box((-1, -1, -1), (1, 2, 3), (16, 24, 32)))
    for q in range(3):
        assert info["h3"][q] == pytest.approx(g.h[q], rel=1e-15)
        assert info["T3"][q] == pytest.approx(g.T[q], rel=1e-15)
    assert info["delta"] == pytest.approx(g.delta, rel=1e-15)
    assert info["R"] == pytest.approx(g.R, rel=1e-15)
    tau_o, _, _ = O.gaussian_sum(1e-12, g.delta, g.R)
    assert info["terms"] == tau_o.size
    with pytest.raises(psn.PsnError):
        p.set_schedule(0, 0)
    assert lib.psn_plan_set_correction(p.handle, psn.CORRECTION_FOURIER) == -1
    assert info["algorithmic_bytes"] == 2 * 8 * 16 * 24 * 32 + 24 * 8 * 16 * 24 * 33 + 8 * 17 * 25 * 33
