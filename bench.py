#!/usr/bin/env python3
"""Throughput of the free-space Poisson solve on one MI355X.

One step = one solve u = U * rho of the n = 512 workload (box [-12, 12]^3,
128-Gaussian seeded mixture, padded 1024^3) through the C ABI: all five pruned
passes, inputs resident in HBM.  Prints ONE JSON line on stdout; progress goes
to stderr.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--n 512] [--no-cpu] [--no-compare]

Reported beside the headline FP32 value: the FP64 and split-precision paths
on the same GPU, each path's max-norm relative error against the FP64 CPU
oracle, the dominant kernel's roofline (algorithmic bytes over its average
duration, measured with HIP events on the solve's stream), and the oracle
itself timed on the host cores as a CPU baseline.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12        # MI355X HBM3E, bytes/s
KERNEL_SOURCES = ("psn_device.h", "psn_passes.h")   # hashed to match a traffic profile to its kernels
PASS_NAMES = ["P1_r2c_axis2", "P2_fwd_axis1", "P3_fwd_mulK_inv_axis0", "P4_inv_axis1", "P5_c2r_axis2"]


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def workload(n):
    import workloads as W
    if n == 512:
        return W.config_n512(), "n=512 on [-12,12]^3, 128-Gaussian seeded mixture (seed 1005), padded 1024^3"
    if n == 256:
        return W.config_n256(), "n=256 on [-10,10]^3, 32-Gaussian seeded mixture (seed 1003), padded 512^3"
    if n == 128:
        return W.config_n128(), "n=128 on [-8,8]^3, 8-Gaussian seeded mixture (seed 1002), padded 256^3"
    raise SystemExit(f"no workload for n={n}")


def host_cpu():
    """Host facts for the CPU baseline: logical CPUs, CPUs this process may use, model name."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count()
    return {"nproc": os.cpu_count(), "affinity": allowed, "model": model}


def oracle_workers():
    """Threads for the oracle's FFTs: the CPUs this process may use, capped at
    the 16 host CPUs that go with one GPU on the measurement box."""
    h = host_cpu()
    return max(1, min(16, h["affinity"] or 1))


def pass_bytes(n, dtype):
    """Algorithmic bytes of P1..P5: each array read and written once.  b1, b2:
    bytes of one complex element of W1 (n^3) and W2 (2 n^3); split precision
    keeps W1 in 12-byte elements and W2 in FP64."""
    bio, b1, b2, bk = {"f32": (4, 8, 8, 4), "f64": (8, 16, 16, 8), "split": (8, 12, 16, 8)}[dtype]
    n3 = float(n) ** 3
    return [(bio + b1) * n3, (b1 + 2 * b2) * n3, 4 * b2 * n3 + bk * (n + 1.0) ** 3, (2 * b2 + b1) * n3,
            (b1 + bio) * n3]


def _sources_digest():
    import hashlib
    try:
        src = b"".join(open(os.path.join(ROOT, "paper_1612_01799_amd", "csrc", f), "rb").read()
                       for f in KERNEL_SOURCES)
    except OSError:
        return None
    return hashlib.sha256(src).hexdigest()[:16]


def _profile_value(path, row_prefix, column):
    """Value of `column` in the row starting with `row_prefix` of a committed
    profile summary, or None if absent or recorded for other kernel sources."""
    if not os.path.exists(path):
        return None
    digest, recorded, header, value = _sources_digest(), None, None, None
    for line in open(path):
        if line.startswith("# kernel sources sha256[:16]"):
            recorded = line.split(":")[-1].strip()
        elif line.startswith("kernel "):
            header = line.split()
        elif header and line.startswith(row_prefix):
            fields = line[len(row_prefix):].split()
            # the kernel name may hold spaces: count columns from the right
            value = float(fields[len(fields) - (len(header) - header.index(column))])
    return value if (value is not None and recorded == digest) else None


def measured_traffic(n, kernel):
    """HBM bytes per launch of the middle pass from the committed rocprofv3 PMC
    summary (copy-calibrated FETCH_SIZE + WRITE_SIZE), or None if there is none
    for this size or the kernel sources changed since it was taken."""
    if kernel != "P3_fwd_mulK_inv_axis0":
        return None
    v = _profile_value(os.path.join(ROOT, "profiles", f"solve_n{n}_f32_hbm_traffic.txt"),
                       f"psn::p3p_conv<{n}, 1,", "total_GB")
    return None if v is None else v * 1e9


def measured_valu(n, kernel):
    """VALU wave-instructions per launch of the middle pass from the committed
    rocprofv3 counter summary (SQ_INSTS_VALU), or None (as measured_traffic)."""
    if kernel != "P3_fwd_mulK_inv_axis0":
        return None
    return _profile_value(os.path.join(ROOT, "profiles", f"solve_n{n}_f32_valu_counters.txt"),
                          f"psn::p3p_conv<{n}, 1,", "valu_insts")


# VALU issue peak: each of the 256 CUs issues one wave64 VALU instruction per
# cycle (4 SIMDs, one every 4 cycles each) at the 2.4 GHz peak clock
VALU_PEAK = 256 * 2.4e9


def alu_roofline(n, kernel, avg_ms):
    """The dominant kernel against its second roof: VALU instruction issue."""
    insts = measured_valu(n, kernel)
    if insts is None:
        return None
    rate = insts / (avg_ms * 1e-3)
    return {"bound": "alu", "kernel": kernel, "achieved": rate / 1e9, "peak": VALU_PEAK / 1e9,
            "unit": "G wave64 VALU instructions/s", "frac": rate / VALU_PEAK, "valu_insts_per_launch": insts,
            "avg_ms": float(avg_ms)}


def time_path(psn, torch, n, L, dtype, rho64, steps, warmup):
    plan = psn.Plan(n, L, 1e-12, dtype).build()
    rho = rho64.to(plan.io_dtype()).contiguous()
    out = torch.empty_like(rho)
    for _ in range(warmup):
        plan.solve(rho, out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        plan.solve(rho, out, stream=stream)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    return plan, rho, out, ms


def bench_batched(psn, torch, np, steps, warmup, with_oracle):
    """64 densities of edges {48,...,160} (h = 0.1), FP32, one captured batch."""
    import workloads as W
    mixes = W.config_batched()
    plans, rhos, cache = [], [], {}
    for mix in mixes:
        n, L = mix.box.n[0], mix.box.b[0]
        if n not in cache:
            cache[n] = psn.Plan(n, L, 1e-12, "f32").build()
        plans.append(cache[n])
        rhos.append(torch.from_numpy(W.mixture_density(mix)).to("cuda", torch.float32))
    outs = [torch.empty_like(r) for r in rhos]
    for _ in range(max(1, warmup)):
        psn.solve_batched(plans, rhos, outs)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        psn.solve_batched(plans, rhos, outs, stream=stream)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    # the same solves one by one on the plans' own workspaces
    tmp = [torch.empty_like(r) for r in rhos]
    for p, r, o in zip(plans, rhos, tmp):
        p.solve(r, o)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(steps):
        for p, r, o in zip(plans, rhos, tmp):
            p.solve(r, o, stream=stream)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_seq = t0.elapsed_time(t1) / steps
    pts = sum(float(p.n) ** 3 for p in plans)
    byts = sum(p.info()["algorithmic_bytes"] for p in plans)
    out = {"workload": "64 seeded 4-Gaussian densities, edges uniform from {48,64,96,128,160}, h = 0.1 "
                       "(seed 1004), FP32, one graph-captured batch",
           "count": len(plans), "grid_points": pts, "ms_per_batch": ms, "value": pts / (ms * 1e-3),
           "unit": "grid pts/s", "hbm_frac": byts / (ms * 1e-3) / HBM_PEAK, "algorithmic_bytes": byts,
           "ms_one_by_one": ms_seq, "max_rel_err_vs_oracle": None}
    if with_oracle:
        import oracle as O
        sym, worst = {}, 0.0
        for mix, u in zip(mixes, outs):
            n, L = mix.box.n[0], mix.box.b[0]
            if n not in sym:
                sym[n] = O.half_spectrum(O.kernel_spectrum(mix.box, 1e-12))
            ref = O.solve(W.mixture_density(mix), sym[n], workers=oracle_workers())
            worst = max(worst, float(np.max(np.abs(u.double().cpu().numpy() - ref)) / np.max(np.abs(ref))))
        out["max_rel_err_vs_oracle"] = worst
    return out


def bench_size(psn, torch, np, n, steps, warmup, with_oracle):
    """F32 and F64 solve times of one more benchmark size (the metric names 256^3 and 512^3)."""
    import workloads as W
    mix, desc = workload(n)
    L = mix.box.b[0]
    rho_np = W.mixture_density(mix)
    rho64 = torch.from_numpy(rho_np).to("cuda")
    out = {"workload": desc, "n": n}
    us = {}
    for dt in ("f32", "f64"):
        p, r, u, ms = time_path(psn, torch, n, L, dt, rho64, steps, warmup)
        out[f"{dt}_ms"] = ms
        out[f"{dt}_value"] = n ** 3 / (ms * 1e-3)
        out[f"{dt}_hbm_frac"] = p.info()["algorithmic_bytes"] / (ms * 1e-3) / HBM_PEAK
        us[dt] = u.double().cpu().numpy()
        del p, r, u
    out["speedup_vs_f64"] = out["f64_ms"] / out["f32_ms"]
    out["max_rel_err_vs_oracle"] = None
    if with_oracle:
        import oracle as O
        ref = O.solve(rho_np, O.half_spectrum(O.kernel_spectrum(mix.box, 1e-12)), workers=oracle_workers())
        out["max_rel_err_vs_oracle"] = {k: float(np.max(np.abs(v - ref)) / np.max(np.abs(ref))) for k, v in us.items()}
    return out


def _timed_solves(torch, plan, rho, out, steps, warmup):
    for _ in range(warmup):
        plan.solve(rho, out)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        plan.solve(rho, out)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def bench_options(psn, torch, np, rho64, steps, warmup):
    """The plan options beyond the cube path, on the benchmark box's spacing:
    a grid with per-axis sizes (512 x 512 x 384, FP32) and the n = 512 solve
    with the near-zone correction by its Fourier series instead of folded."""
    import workloads as W
    out = {}
    n3, h = (512, 512, 384), 24.0 / 511
    a = tuple(-0.5 * h * (q - 1) for q in n3)
    b = tuple(0.5 * h * (q - 1) for q in n3)
    box = W.Box(a, b, n3)
    half = min(b)
    mix = W.draw_mixture(1006, 64, -0.5 * half, 0.5 * half, 0.3, 2.0, 0.5, 1.5, box)
    plan = psn.Plan(n3, box=(a, b), tol=1e-12, dtype="f32").build()
    rho = torch.from_numpy(W.mixture_density(mix)).to("cuda", torch.float32)
    u = torch.empty_like(rho)
    ms = _timed_solves(torch, plan, rho, u, steps, warmup)
    out["grid_per_axis"] = {
        "workload": "512 x 512 x 384 grid, h = 24/511, 64-Gaussian seeded mixture (seed 1006), FP32",
        "ms": ms, "value": float(np.prod(n3)) / (ms * 1e-3),
        "hbm_frac": plan.info()["algorithmic_bytes"] / (ms * 1e-3) / HBM_PEAK}
    del plan, rho, u
    plan = psn.Plan(512, 12.0, 1e-12, "f32", correction="fourier").build()
    rho = rho64.to(torch.float32).contiguous()
    u = torch.empty_like(rho)
    ms = _timed_solves(torch, plan, rho, u, steps, warmup)
    out["fourier_correction"] = {"workload": "the n=512 benchmark workload, FP32, correction by the Fourier series",
                                 "ms": ms, "value": 512.0 ** 3 / (ms * 1e-3)}
    del plan, rho, u
    return out


def kernel_build_times(psn, torch, n, reps=3):
    """Wall time of psn_kernel_build (setup: mode integrals, correction
    constants, octant assembly, workspace allocation) on the benchmark box."""
    mix, desc = workload(n)
    out = {"metric": "kernel build (setup) wall time", "unit": "ms", "workload": desc, "n": n}
    torch.cuda.init()
    for dt in ("f32", "f64"):
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            plan = psn.Plan(n, mix.box.b[0], 1e-12, dt).build()
            torch.cuda.synchronize()
            ts.append(1e3 * (time.perf_counter() - t))
            del plan
        out[f"{dt}_ms"] = ts
        log(f"kernel build {dt}: " + ", ".join(f"{v:.1f}" for v in ts) + " ms")
    return out


def radix16_probe():
    """Radix-16 DFTs per second: VALU butterflies vs FP32 MFMA (built by build.py)."""
    import subprocess
    exe = os.path.join(ROOT, "paper_1612_01799_amd", "dft16_valu_vs_mfma")
    if not os.path.exists(exe):
        return None
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    out = {}
    for tok in r.stdout.split():
        k, _, v = tok.partition("=")
        try:
            out[k] = float(v)
        except ValueError:
            out[k] = v
    if r.returncode == 0 and "valu_dft16_per_s" in out:
        out["valu_over_mfma"] = out["valu_dft16_per_s"] / out["mfma_dft16_per_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 and split paths")
    ap.add_argument("--no-batched", action="store_true", help="skip the mixed-size batched workload")
    ap.add_argument("--no-options", action="store_true",
                    help="skip the per-axis grid and Fourier-series correction timings")
    ap.add_argument("--extra-n", type=int, default=256, help="second benchmark size (0 = none)")
    ap.add_argument("--kernel-build", action="store_true",
                    help="only time psn_kernel_build (the setup phase) for the benchmark box, FP32 and FP64, "
                         "with the schedule autotuner off, and print one JSON line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device tensor copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures exactly one GPU; --gpus {args.gpus} is not supported "
              "(independent solves shard across GPUs with no communication between them)",
              file=sys.stderr)
        sys.exit(2)

    if args.kernel_build:
        os.environ["PSN_TUNE"] = "0"   # read by the library at build time
    import numpy as np
    import torch

    import paper_1612_01799_amd as psn
    import workloads as W

    n = args.n
    if args.kernel_build:
        print(json.dumps(kernel_build_times(psn, torch, n)), flush=True)
        return
    mix, desc = workload(n)
    L = mix.box.b[0]
    log(f"generating density n={n}")
    rho_np = W.mixture_density(mix)
    rho64 = torch.from_numpy(rho_np).to("cuda")
    torch.cuda.synchronize()

    log("timing f32 path")
    plan32, rho32, u32, ms32 = time_path(psn, torch, n, L, "f32", rho64, args.steps, args.warmup)
    info32 = plan32.info()
    log(f"f32: {ms32:.3f} ms/solve")

    # dominant kernel: per-pass HIP events on the solve's stream
    reps = max(5, args.steps // 2)
    passes = np.zeros(5)
    for _ in range(reps):
        passes += plan32.solve_timed(rho32, u32)
    passes /= reps
    pb = pass_bytes(n, "f32")
    dom = int(np.argmax(passes))
    achieved = pb[dom] / (passes[dom] * 1e-3)
    log("pass ms: " + ", ".join(f"{PASS_NAMES[i]}={passes[i]:.3f}" for i in range(5)))

    extra = {}
    outs = {"f32": u32}
    if not args.no_compare:
        for dt in ("f64", "split"):
            log(f"timing {dt} path")
            p, r, u, ms = time_path(psn, torch, n, L, dt, rho64, max(3, args.steps // 2), args.warmup)
            pm = np.zeros(5)
            for _ in range(3):
                pm += p.solve_timed(r, u)
            pm /= 3
            extra[dt] = {"ms_per_step": ms, "value": n ** 3 / (ms * 1e-3),
                         "hbm_frac_whole_solve": p.info()["algorithmic_bytes"] / (ms * 1e-3) / HBM_PEAK,
                         "pass_ms": {PASS_NAMES[i]: float(pm[i]) for i in range(5)}}
            log(f"{dt} pass ms: " + ", ".join(f"{PASS_NAMES[i]}={pm[i]:.3f}" for i in range(5)))
            outs[dt] = u
            log(f"{dt}: {ms:.3f} ms/solve")
            del p, r
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst
    u_host = {k: v.double().cpu().numpy() for k, v in outs.items()}
    del outs
    torch.cuda.synchronize()

    cpu = None
    errs = {}
    if not args.no_cpu:
        import oracle as O
        workers = oracle_workers()
        host = host_cpu()
        log(f"oracle kernel spectrum (setup, untimed), {workers} threads; host {host}")
        H = O.half_spectrum(O.kernel_spectrum(mix.box, 1e-12))
        reps = 3
        log(f"oracle solve (timed, {reps} runs)")
        times = []
        for _ in range(reps):
            t = time.perf_counter()
            uref = O.solve(rho_np, H, workers=workers)
            times.append(time.perf_counter() - t)
        dt_cpu = float(np.median(times))
        del H
        cpu = {"value": n ** 3 / dt_cpu, "unit": "grid pts/s", "cores": workers, "kind": "oracle",
               "sample": f"{reps} full FP64 oracle solves of the same n={n} workload (unpruned padded "
                         f"rfftn/irfftn, scipy.fft with {workers} workers; kernel spectrum built beforehand), "
                         f"median {dt_cpu:.2f} s of " + ", ".join(f"{v:.2f}" for v in times) + " s",
               "host_nproc": host["nproc"], "host_cpus_allowed": host["affinity"], "host_cpu_model": host["model"],
               "workers_rule": "min(16, CPUs allowed): the host CPU share of one GPU on the measurement box"}
        scale = float(np.max(np.abs(uref)))
        for k, v in u_host.items():
            errs[k] = float(np.max(np.abs(v - uref)) / scale)
        log("oracle errors: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()))

    second = None
    if args.extra_n and args.extra_n != n:
        log(f"timing n={args.extra_n}")
        second = bench_size(psn, torch, np, args.extra_n, args.steps, args.warmup, not args.no_cpu)
        log(f"n={args.extra_n}: f32 {second['f32_ms']:.3f} ms, f64 {second['f64_ms']:.3f} ms, "
            f"err {second['max_rel_err_vs_oracle']}")

    batched = None
    if not args.no_batched:
        log("timing the batched mixed-size workload")
        batched = bench_batched(psn, torch, np, max(3, args.steps // 2), args.warmup, not args.no_cpu)
        log(f"batched: {batched['ms_per_batch']:.3f} ms/batch ({batched['ms_one_by_one']:.3f} ms one by one), "
            f"err {batched['max_rel_err_vs_oracle']}")

    options = None
    if not args.no_options and n == 512:
        log("timing the plan options (per-axis grid, Fourier-series correction)")
        options = bench_options(psn, torch, np, rho64, max(3, args.steps // 4), max(1, args.warmup))
        log(f"options: {options}")

    log("radix-16 DFT: VALU butterflies vs FP32 MFMA")
    r16 = radix16_probe()
    log(f"radix-16: {r16}")

    value = n ** 3 / (ms32 * 1e-3)
    line = {
        "metric": "grid pts/s per solve at 256^3/512^3 vs FP64 path, max rel err, % HBM peak",
        "value": value,
        "unit": "grid pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "padded": 2 * n, "path": "f32", "tol": 1e-12,
                   "schedule": list(info32["schedule"]), "tuned": bool(info32["tuned"])},
        "roofline_alu": alu_roofline(n, PASS_NAMES[dom], passes[dom]),
        "roofline": {"bound": "hbm", "kernel": PASS_NAMES[dom], "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": measured_traffic(n, PASS_NAMES[dom]),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes_per_launch": pb[dom], "avg_ms": float(passes[dom])},
        "pass_ms": {PASS_NAMES[i]: float(passes[i]) for i in range(5)},
        "hbm_frac_whole_solve": info32["algorithmic_bytes"] / (ms32 * 1e-3) / HBM_PEAK,
        "algorithmic_bytes_per_solve": info32["algorithmic_bytes"],
        "cpu_baseline": cpu,
        "f64_path": extra.get("f64"),
        "split_path": extra.get("split"),
        "speedup_vs_f64": (extra["f64"]["ms_per_step"] / ms32) if "f64" in extra else None,
        "max_rel_err_vs_oracle": errs or None,
        f"n{args.extra_n}": second,
        "batched": batched,
        "plan_options": options,
        "radix16_valu_vs_mfma": r16,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
