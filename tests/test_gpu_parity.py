"""GPU path (through the C ABI) against the FP64 CPU oracle, element by element.

Tolerances (max-norm relative error against the oracle): FP64 1e-12,
split precision 1e-10, FP32 1e-5.
"""
import math

import numpy as np
import pytest

import oracle as O
import paper_cases as PC
import workloads as W
from gpu_common import TOL, gpu_solve, max_rel, oracle_octant, oracle_symbol, torch_cuda

pytestmark = pytest.mark.gpu
psn = pytest.importorskip("paper_1612_01799_amd")

SIZES = [8, 12, 16, 24, 32, 48, 64, 96, 128, 160, 162, 192, 320, 384]


def _mix(n, L, seed):
    return W.mixture_density(W.draw_mixture(seed, 5, -L / 3, L / 3, 0.25 * L / 2, 0.45 * L / 2, 0.5, 1.5,
                                            W.Box.cube(L, n)))


@pytest.mark.parametrize("n", [8, 16, 32, 48, 128])
@pytest.mark.parametrize("dtype", ["f64", "f32", "split"])
def test_kernel_spectrum_matches_oracle(n, dtype):
    torch_cuda()
    L = 2.0 + 0.1 * n
    plan = psn.Plan(n, L, 1e-12, dtype).build()
    K = plan.kernel_octant()
    Ko = oracle_octant(n, L)
    tol = 1e-13 if dtype != "f32" else 2e-7
    assert np.max(np.abs(K - Ko)) <= tol * abs(Ko[0, 0, 0])
    info = plan.info()
    ks = O.kernel_spectrum(W.Box.cube(L, n), 1e-12)
    _check_correction_constants(info, ks)


def _check_correction_constants(info, ks):
    """C0 = delta^2/2 - 4 pi sum_j w_j I2 and C2 = delta^4/4 - 4 pi sum_j w_j I4
    are differences of nearly equal terms, so their rounding is relative to
    delta^2/2 and delta^4/4, not to C0 and C2 themselves."""
    d = info["delta"]
    assert abs(info["C0"] - ks.C0) <= 1e-14 * d ** 2
    assert abs(info["C2"] - ks.C2) <= 1e-14 * d ** 4


@pytest.mark.parametrize("dtype", ["f64", "f32", "split"])
def test_box_kernel_and_solve_match_oracle(dtype):
    """Rectangular box [-3,2] x [-2,3.5] x [-1,5]: per-axis spacing and modes."""
    torch = torch_cuda()
    n = 32
    box = W.Box((-3.0, -2.0, -1.0), (2.0, 3.5, 5.0), (n, n, n))
    plan = psn.Plan(n, box=(box.a, box.b), tol=1e-12, dtype=dtype).build()
    ks = O.kernel_spectrum(box, 1e-12)
    K = plan.kernel_octant()
    tol = 1e-13 if dtype != "f32" else 2e-7
    assert np.max(np.abs(K - ks.octant)) <= tol * abs(ks.octant[0, 0, 0])
    mix = W.draw_mixture(41, 4, -0.3, 0.6, 0.35, 0.6, 0.5, 1.5, box)
    rho = W.mixture_density(mix)
    ref = O.solve(rho, O.half_spectrum(ks))
    u = gpu_solve(psn, torch, n, None, dtype, rho, plan=plan)
    assert max_rel(u, ref) <= TOL[dtype]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dtype", ["f64", "f32", "split"])
def test_solve_matches_oracle(n, dtype):
    torch = torch_cuda()
    print(f"case n={n} dtype={dtype}", flush=True)
    L = 3.0
    rho = _mix(n, L, 100 + n)
    ref = O.solve(rho, oracle_symbol(n, L))
    u = gpu_solve(psn, torch, n, L, dtype, rho)
    assert max_rel(u, ref) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32", "split"])
def test_random_density_all_frequencies(dtype):
    """White-noise density excites every frequency, including the packed
    DC/Nyquist column and the self-conjugate rows of the middle pass."""
    torch = torch_cuda()
    n, L = 24, 1.7
    rho = np.random.default_rng(5).standard_normal((n, n, n))
    ref = O.solve(rho, oracle_symbol(n, L))
    u = gpu_solve(psn, torch, n, L, dtype, rho)
    err = max_rel(u, ref)
    print(f"white noise n={n} {dtype}: max rel err {err:.3e}", flush=True)
    assert err <= TOL[dtype]


def _gpu_entries():
    g = PC.load()
    return g["digits"] + g["three_digits"]


@pytest.mark.parametrize("entry", _gpu_entries(), ids=[PC.name(e) for e in _gpu_entries()])
def test_paper_tables_on_gpu_fp64(entry):
    """The printed E of Tables 1-7 (cubes and rectangular boxes), reproduced by
    the FP64 GPU path."""
    torch = torch_cuda()
    box, rho, ustar = PC.case(entry)
    plan = psn.Plan(box.n[0], box=(box.a, box.b), tol=entry.get("eps", 1e-12), dtype="f64").build()
    u = gpu_solve(psn, torch, box.n[0], None, "f64", rho, plan=plan)
    E = O.error_E(u, ustar)
    digits = 4 if entry in PC.load()["digits"] else 3
    assert abs(E - entry["E"]) <= 0.5 * 10 ** (math.floor(math.log10(entry["E"])) - (digits - 1)) * 1.0001


@pytest.mark.parametrize("entry", PC.load()["bounds"], ids=[PC.name(e) for e in PC.load()["bounds"]])
def test_paper_converged_rows_on_gpu_fp64(entry):
    """Converged rows (Table 1 at 64^3, Table 6 up to 162^3 on its rectangular
    box): the FP64 GPU path stays within the printed bound and equals the
    oracle's result."""
    torch = torch_cuda()
    box, rho, ustar = PC.case(entry)
    eps = entry.get("eps", 1e-12)
    plan = psn.Plan(box.n[0], box=(box.a, box.b), tol=eps, dtype="f64").build()
    u = gpu_solve(psn, torch, box.n[0], None, "f64", rho, plan=plan)
    assert O.error_E(u, ustar) <= entry["max"]
    ref = O.solve(rho, O.half_spectrum(O.kernel_spectrum(box, eps)))
    assert max_rel(u, ref) <= TOL["f64"]


def test_single_gaussian_closed_form_fp64():
    torch = torch_cuda()
    mix = W.config_single()
    u = gpu_solve(psn, torch, 32, 6.0, "f64", W.mixture_density(mix))
    assert O.error_E(u, O.analytic.mixture(mix)) <= 1e-10


@pytest.mark.parametrize("dtype", ["f64", "f32", "split"])
def test_n128_mixture(dtype):
    torch = torch_cuda()
    mix = W.config_n128()
    rho = W.mixture_density(mix)
    ref = O.solve(rho, oracle_symbol(128, 8.0))
    u = gpu_solve(psn, torch, 128, 8.0, dtype, rho)
    assert max_rel(u, ref) <= TOL[dtype]
    if dtype == "f64":
        assert O.error_E(u, O.analytic.mixture(mix)) <= 1e-10


@pytest.mark.parametrize("dtype", ["f64", "f32", "split"])
def test_n256_mixture(dtype):
    torch = torch_cuda()
    mix = W.config_n256()
    rho = W.mixture_density(mix)
    ref = _n256_ref()
    u = gpu_solve(psn, torch, 256, 10.0, dtype, rho)
    assert max_rel(u, ref) <= TOL[dtype]


_cache = {}


def _n256_ref():
    if "n256" not in _cache:
        mix = W.config_n256()
        _cache["n256"] = O.solve(W.mixture_density(mix), oracle_symbol(256, 10.0))
    return _cache["n256"]


def test_zero_density_gives_zero():
    torch = torch_cuda()
    for dt in ["f64", "f32", "split"]:
        u = gpu_solve(psn, torch, 16, 1.0, dt, np.zeros((16, 16, 16)))
        assert np.all(u == 0)


def test_in_place_and_plan_reuse_and_determinism():
    torch = torch_cuda()
    n, L = 32, 2.5
    plan = psn.Plan(n, L, 1e-12, "f32").build()
    sym = oracle_symbol(n, L)
    for seed in (1, 2):
        rho_np = _mix(n, L, seed)
        rho = torch.from_numpy(rho_np).to("cuda", torch.float32)
        a = plan.solve(rho)
        b = plan.solve(rho)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        c = rho.clone()
        plan.solve(c, out=c)
        torch.cuda.synchronize()
        assert torch.equal(a, c)
        assert max_rel(a.double().cpu().numpy(), O.solve(rho_np, sym)) <= TOL["f32"]


def test_side_stream():
    torch = torch_cuda()
    n, L = 32, 2.5
    plan = psn.Plan(n, L, 1e-12, "f64").build()
    rho_np = _mix(n, L, 3)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        rho = torch.from_numpy(rho_np).to("cuda")
        u = plan.solve(rho, stream=s)
    s.synchronize()
    assert max_rel(u.cpu().numpy(), O.solve(rho_np, oracle_symbol(n, L))) <= TOL["f64"]


def test_batched_full_mixed_size_workload():
    """The whole mixed-size workload: 64 seeded densities with edges drawn from
    {48, 64, 96, 128, 160} (h = 0.1), FP32, in ONE batched call (the launch
    configuration the benchmark times); every problem against the oracle."""
    torch = torch_cuda()
    mixes = W.config_batched()
    assert len(mixes) == 64 and {m.box.n[0] for m in mixes} == set(W.BATCH_EDGES)
    plans, rhos, refs = _batch_case(torch, mixes, "f32")
    outs = psn.solve_batched(plans, rhos)
    torch.cuda.synchronize()
    errs = [max_rel(u.double().cpu().numpy(), ref) for u, ref in zip(outs, refs)]
    print(f"64-problem batch: worst max rel err {max(errs):.3e}", flush=True)
    assert max(errs) <= TOL["f32"]


def test_batched_odd_sizes_f32_and_split():
    """n = 96 (factor 3) and n = 160 (factor 5) inside one batch graph, in FP32
    and in split precision, beside a power-of-two size."""
    torch = torch_cuda()
    mixes = W.config_batched(seed=2024, count=40)
    pick = []
    for n in (96, 160, 64):
        pick += [m for m in mixes if m.box.n[0] == n][:2]
    assert {m.box.n[0] for m in pick} == {96, 160, 64}
    p32, r32, ref32 = _batch_case(torch, pick, "f32")
    psp, rsp, refsp = _batch_case(torch, pick, "split")
    outs = psn.solve_batched(p32 + psp, r32 + rsp)
    torch.cuda.synchronize()
    k = len(pick)
    for i, (u, ref) in enumerate(zip(outs, ref32 + refsp)):
        dt = "f32" if i < k else "split"
        err = max_rel(u.double().cpu().numpy(), ref)
        print(f"odd-size batch entry {i} n={pick[i % k].box.n[0]} {dt}: {err:.3e}", flush=True)
        assert err <= TOL[dt]


def test_batched_mixed_sizes():
    torch = torch_cuda()
    mixes = W.config_batched(count=10)
    plans, rhos, refs = [], [], []
    cache = {}
    for mix in mixes:
        n = mix.box.n[0]
        L = mix.box.b[0]
        if n not in cache:
            cache[n] = psn.Plan(n, L, 1e-12, "f32").build()
        plans.append(cache[n])
        rho = W.mixture_density(mix)
        rhos.append(torch.from_numpy(rho).to("cuda", torch.float32))
        refs.append(O.solve(rho, oracle_symbol(n, L)))
    outs = psn.solve_batched(plans, rhos)
    torch.cuda.synchronize()
    for u, ref in zip(outs, refs):
        assert max_rel(u.double().cpu().numpy(), ref) <= TOL["f32"]
    assert psn.solve_batched([], []) == []


_cache512 = {}


def _ks512():
    if "ks" not in _cache512:
        _cache512["ks"] = O.kernel_spectrum(W.config_n512().box, 1e-12)
    return _cache512["ks"]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_kernel_spectrum_n512_matches_oracle(dtype):
    """The whole (n+1)^3 octant of the n = 512 benchmark box against the
    oracle's FP64 G-tensor plus correction symbol."""
    torch_cuda()
    ks = _ks512()
    plan = psn.Plan(512, 12.0, 1e-12, dtype).build()
    K = plan.kernel_octant()
    tol = 1e-13 if dtype == "f64" else 2e-7
    err = float(np.max(np.abs(K - ks.octant)))
    print(f"n=512 {dtype} kernel: max abs err / K(0) = {err / abs(ks.octant[0, 0, 0]):.3e}", flush=True)
    assert err <= tol * abs(ks.octant[0, 0, 0])
    _check_correction_constants(plan.info(), ks)
    # symmetric in (k0, k1) on a cube, exactly
    assert np.array_equal(K, np.transpose(K, (1, 0, 2)))


@pytest.mark.parametrize("dtype", ["f32", "f64", "split"])
def test_n512_mixture_full_size(dtype):
    """n = 512 on [-12,12]^3 (the benchmark workload, 128 Gaussians), full
    oracle solve (padded 1024^3 in FP64 on the host), same launch
    configuration as the benchmark."""
    torch = torch_cuda()
    mix = W.config_n512()
    if "ref" not in _cache512:
        rho = W.mixture_density(mix)
        _cache512["rho"] = rho
        _cache512["ref"] = O.solve(rho, O.half_spectrum(_ks512()))
    u = gpu_solve(psn, torch, 512, 12.0, dtype, _cache512["rho"])
    assert max_rel(u, _cache512["ref"]) <= TOL[dtype]


def _batch_case(torch, mixes, dtype):
    plans, rhos, refs, cache = [], [], [], {}
    for mix in mixes:
        n, L = mix.box.n[0], mix.box.b[0]
        if (n, L) not in cache:
            cache[(n, L)] = psn.Plan(n, L, 1e-12, dtype).build()
        plans.append(cache[(n, L)])
        rho = W.mixture_density(mix)
        rhos.append(torch.from_numpy(rho).to("cuda", plans[-1].io_dtype()))
        refs.append(O.solve(rho, oracle_symbol(n, L)))
    return plans, rhos, refs


def test_batched_repeated_plan_graph_replay_and_chunking():
    """40 problems of one size on ONE plan (more than one launch table of 32),
    replayed from the captured graph with new input values."""
    torch = torch_cuda()
    n, L = 32, 2.5
    plan = psn.Plan(n, L, 1e-12, "f32").build()
    sym = oracle_symbol(n, L)
    rng = np.random.default_rng(17)
    rhos_np = [_mix(n, L, 200 + i) for i in range(40)]
    rhos = [torch.from_numpy(r).to("cuda", torch.float32) for r in rhos_np]
    outs = [torch.empty_like(r) for r in rhos]
    psn.solve_batched([plan] * 40, rhos, outs)
    torch.cuda.synchronize()
    for u, r in zip(outs, rhos_np):
        assert max_rel(u.double().cpu().numpy(), O.solve(r, sym)) <= TOL["f32"]
    # same pointers, new values: the replayed graph must see them
    for i, r in enumerate(rhos):
        rhos_np[i] = rng.standard_normal((n, n, n)) * np.exp(-np.arange(n) / 8.0)[None, None, :]
        r.copy_(torch.from_numpy(rhos_np[i]))
    psn.solve_batched([plan] * 40, rhos, outs)
    torch.cuda.synchronize()
    worst = max(max_rel(u.double().cpu().numpy(), O.solve(r, sym)) for u, r in zip(outs, rhos_np))
    print(f"graph replay with new values: worst max rel err {worst:.3e}", flush=True)
    assert worst <= TOL["f32"]


def test_batched_mixed_precisions_and_sizes():
    torch = torch_cuda()
    mixes = W.config_batched(seed=77, count=6)
    p32, r32, ref32 = _batch_case(torch, mixes[:3], "f32")
    p64, r64, ref64 = _batch_case(torch, mixes[3:], "f64")
    outs = psn.solve_batched(p32 + p64, r32 + r64)
    torch.cuda.synchronize()
    for u, ref in zip(outs[:3], ref32):
        assert max_rel(u.double().cpu().numpy(), ref) <= TOL["f32"]
    for u, ref in zip(outs[3:], ref64):
        assert max_rel(u.cpu().numpy(), ref) <= TOL["f64"]


def test_batched_after_plan_destroyed():
    """A captured batch must not outlive the plans it references."""
    torch = torch_cuda()
    n, L = 16, 1.5
    rho_np = _mix(n, L, 9)
    rho = torch.from_numpy(rho_np).to("cuda", torch.float64)
    out = torch.empty_like(rho)
    for _ in range(3):
        plan = psn.Plan(n, L, 1e-12, "f64").build()
        psn.solve_batched([plan], [rho], [out])
        torch.cuda.synchronize()
        assert max_rel(out.cpu().numpy(), O.solve(rho_np, oracle_symbol(n, L))) <= TOL["f64"]
        plan.close()


@pytest.mark.parametrize("n", [24, 48, 96, 128, 160, 162, 256])
@pytest.mark.parametrize("dtype", ["f32", "f64", "split"])
def test_every_schedule_candidate(n, dtype):
    """All compiled tile candidates of the strided passes give the oracle's result."""
    torch = torch_cuda()
    L = 2.0 + n / 64.0
    rho = _mix(n, L, 300 + n)
    ref = O.solve(rho, oracle_symbol(n, L))
    plan = psn.Plan(n, L, 1e-12, dtype).build()
    info = plan.info()
    assert info["tuned"] == 1 and all(0 <= v < 4 for v in info["schedule"])
    for s in [(0, 0), (1, 1), (2, 2), (3, 3), (1, 2), (2, 0), (3, 0), (0, 3)]:
        plan.set_schedule(*s)
        u = gpu_solve(psn, torch, n, L, dtype, rho, plan=plan)
        assert max_rel(u, ref) <= TOL[dtype], s


def test_every_schedule_candidate_n512():
    torch = torch_cuda()
    mix = W.config_n512()
    if "ref" not in _cache512:
        rho = W.mixture_density(mix)
        _cache512["rho"] = rho
        _cache512["ref"] = O.solve(rho, O.half_spectrum(_ks512()))
    plan = psn.Plan(512, 12.0, 1e-12, "f32").build()
    for s in [(0, 0), (1, 1), (2, 2), (3, 3)]:
        plan.set_schedule(*s)
        u = gpu_solve(psn, torch, 512, 12.0, "f32", _cache512["rho"], plan=plan)
        assert max_rel(u, _cache512["ref"]) <= TOL["f32"], s


@pytest.mark.parametrize("n", [96, 128])
@pytest.mark.parametrize("dtype", ["f32", "f64", "split"])
def test_bitwise_determinism_every_schedule(n, dtype):
    """Repeated solves give bitwise-equal results under every schedule the
    autotuner may pick (a race in an LDS exchange or a missing barrier would
    show up as run-to-run differences)."""
    torch = torch_cuda()
    L = 2.0 + n / 64.0
    rho_np = _mix(n, L, 500 + n)
    plan = psn.Plan(n, L, 1e-12, dtype).build()
    rho = torch.from_numpy(rho_np).to("cuda", plan.io_dtype())
    for v24 in range(4):
        for v3 in range(4):
            plan.set_schedule(v24, v3)
            a = plan.solve(rho)
            b = plan.solve(rho)
            c = plan.solve(rho)
            torch.cuda.synchronize()
            assert torch.equal(a, b) and torch.equal(a, c), (v24, v3)


def test_binding_rejects_bad_tensors_before_launch():
    """Wrong device, dtype, shape or layout raises ValueError in the binding;
    nothing reaches the kernels."""
    torch = torch_cuda()
    n = 16
    plan = psn.Plan(n, 1.5, 1e-12, "f32").build()
    assert plan.device() == torch.cuda.current_device()
    rho = torch.zeros((n, n, n), device="cuda", dtype=torch.float32)
    bad_outs = [torch.zeros((n, n, n), dtype=torch.float32),                       # host memory
                torch.zeros((n, n, n), device="cuda", dtype=torch.float64),        # wrong dtype
                torch.zeros((n, n, 2 * n), device="cuda", dtype=torch.float32)[:, :, ::2],  # strided
                torch.zeros((n, n, n + 1), device="cuda", dtype=torch.float32)]    # wrong shape
    for o in bad_outs:
        with pytest.raises(ValueError):
            plan.solve(rho, out=o)
        with pytest.raises(ValueError):
            psn.solve_batched([plan], [rho], [o])
    with pytest.raises(ValueError):
        plan.solve(rho.double())
    with pytest.raises(ValueError):
        psn.solve_batched([plan], [rho.double()])
    with pytest.raises(ValueError):
        psn.solve_batched([plan], [rho], [])


def test_tune_cache_file(tmp_path, monkeypatch):
    """PSN_TUNE_CACHE: a recorded schedule is taken without timing; a plan
    whose (n, precision) has no record appends one."""
    torch_cuda()
    path = tmp_path / "tune.txt"
    path.write_text("32 1 2 1\n")
    monkeypatch.setenv("PSN_TUNE_CACHE", str(path))
    plan = psn.Plan(32, 2.5, 1e-12, "f32").build()
    info = plan.info()
    assert info["schedule"] == (2, 1) and info["tuned"] == 1
    plan2 = psn.Plan(16, 1.5, 1e-12, "f64").build()
    recs = [tuple(int(v) for v in line.split()) for line in path.read_text().split("\n") if line.strip()]
    assert (16, 0) + tuple(plan2.info()["schedule"]) in recs
