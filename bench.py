"""Benchmark: grid points/s of the sphere GRF sampler on one MI355X.

A step is one pass of the whole sampling path -- the ring recursion with fused Philox
normals for every (field, mode, part, hemisphere) chain, then the in-place C2R FFT of
every ring -- over one call of 8 fields on the 4096 x 8192 grid (order 2,
C_l = (l(l+1) + 50^2)^-2, ell_max 4095, FP64 setup, FP32 sampling).  Setup is outside the
timed region; inputs (the factors) are resident in HBM when timing starts.

Prints one JSON line.  Besides the contract fields it carries the FP64 plain path on the
same workload (the speedup of the FP32 path over it), per-kernel times, the roofline of
the dominant kernel and the CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("rng.h", "device_path.h", "sample.hip", "smf_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1709_10314_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def time_calls(fn, steps, warmup):
    """Average ms per call of fn() over `steps` calls after `warmup`, HIP events on the
    current stream (the stream the library launches on), plus wall-clock ms."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return e0.elapsed_time(e1) / steps, wall


def measured_traffic(kernel):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, if they were taken on
    the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(cfg, rings):
    """The FP64 oracle (chains + naive DFT) on `rings` rings around the equator of one
    field of the workload; its factor sets are built first, untimed."""
    import numpy as np

    import oracle
    from paper_1709_10314_amd import workloads

    n, nphi, order, lmax = cfg["n_theta"], cfg["n_phi"], cfg["order"], cfg["ell_max"]
    s = n // 2 - 1
    sets = rings // 2 + 1
    C = oracle.spectrum(workloads.kappas(cfg), lmax)
    t0 = time.perf_counter()
    A, B = oracle.setup(order, C, n, nphi, sets=sets)
    t_setup = time.perf_counter() - t0
    r0, r1 = s - rings // 2 + 1, s + rings // 2 + 1
    t0 = time.perf_counter()
    g = oracle.sample_modes(order, n, A, B, cfg["seed"], 1, sets=sets)
    T = oracle.dft(g, nphi, r0, r1)
    dt = time.perf_counter() - t0
    assert np.all(np.isfinite(T))
    pts = rings * nphi
    return {"value": pts / dt, "unit": "grid points/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": (f"{cfg['name']}: field 1, the {rings} rings around the equator (all "
                       f"{lmax + 1} modes), chains + naive DFT in FP64; setup of the {sets} "
                       f"factor sets they need ({t_setup:.1f} s) not timed"),
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-rings", type=int, default=96)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (calibrates rocprofv3 FETCH/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the sampler shards by whole fields with no exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("RANK", "0")) != 0:
        return

    import torch

    if args.copy_calibration:
        n = 1 << 28                                   # 2^28 floats = 1 GiB each way
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": 4 * n, "launches": 3}), flush=True)
        return

    from paper_1709_10314_amd import Plan, workloads

    cfg = workloads.PRECISION_4096
    n, nphi, order, lmax, count, seed = (cfg[k] for k in ("n_theta", "n_phi", "order", "ell_max",
                                                           "count", "seed"))
    pts = count * n * nphi
    torch.cuda.set_device(0)
    log(f"setup {cfg['name']} (fp32)")
    t0 = time.perf_counter()
    plan = Plan(order, n, nphi, lmax, kappa=workloads.kappas(cfg), precision="fp32")
    setup_s = time.perf_counter() - t0
    out = plan.empty(count)
    log(f"  setup {setup_s:.2f} s; timing {args.steps} steps")
    ms_step, wall_step = time_calls(lambda: plan.sample(seed, count, out), args.steps, args.warmup)
    log(f"  {ms_step:.3f} ms/step ({pts / ms_step * 1e3:.3e} pts/s)")
    ms_rec, _ = time_calls(lambda: plan.sample_modes(seed, count, out), args.steps, args.warmup)
    ms_fft = max(ms_step - ms_rec, 1e-9)
    log(f"  recursion {ms_rec:.3f} ms, fft {ms_fft:.3f} ms")
    m_top = plan.m_top
    n_sets = plan.n_sets
    plan.close()
    del out
    torch.cuda.empty_cache()

    fp64 = None
    if not args.no_fp64:
        log("setup fp64 plain path on the same workload")
        plan64 = Plan(order, n, nphi, lmax, kappa=workloads.kappas(cfg), precision="fp64")
        out64 = plan64.empty(count)
        ms64, _ = time_calls(lambda: plan64.sample(seed, count, out64), max(args.steps // 2, 3), 2)
        plan64.close()
        del out64
        torch.cuda.empty_cache()
        fp64 = {"value": pts / ms64 * 1e3, "unit": "grid points/s", "ms_per_step": ms64}
        log(f"  fp64 {ms64:.3f} ms/step")

    # algorithmic bytes per launch (see the design notes for the per-unit figures)
    vals_per_rec = order * order + order * (order + 1) // 2
    fac_bytes = n_sets * (m_top + 1) * vals_per_rec * 4
    g_bytes = count * n * (nphi // 2) * 8
    kernels = {
        "recursion": {"ms": ms_rec, "alg_bytes": fac_bytes + g_bytes},
        "c2r_fft": {"ms": ms_fft, "alg_bytes": 2 * count * n * nphi * 4},
    }
    for k, v in kernels.items():
        v["alg_GBs"] = v["alg_bytes"] / (v["ms"] * 1e-3) / 1e9
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    kd = kernels[dom]
    traffic = measured_traffic(dom)
    roofline = {"bound": "hbm", "achieved": kd["alg_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": kd["alg_GBs"] / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                "path_alg_GBs": (fac_bytes + g_bytes + 2 * count * n * nphi * 4) / (ms_step * 1e-3) / 1e9}

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on {args.cpu_rings} rings")
        cpu = cpu_baseline(cfg, args.cpu_rings)
        log(f"  {cpu['value']:.3e} pts/s on {cpu['cores']} threads in {cpu['seconds']:.1f} s")

    line = {
        "metric": "grid points/s (FP32 batched vs FP64 plain) at 4096x8192; % HBM roofline",
        "value": pts / ms_step * 1e3,
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "wall_ms_per_step": wall_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "n_theta": n, "n_phi": nphi, "order": order,
                   "kappa": cfg["kappa"], "ell_max": lmax, "fields": count, "seeds": f"{seed}..{seed + count - 1}",
                   "setup": "fp64 on GPU (untimed)", "setup_s": setup_s},
        "roofline": roofline,
        "kernels": kernels,
        "fp64_plain": fp64,
        "speedup_fp32_vs_fp64": (fp64["ms_per_step"] / ms_step) if fp64 else None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
