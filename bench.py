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
# Lane-FMAs per second of the unpacked FP32 FMA the library is built with (packed FP32 is
# switched off): 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz, i.e. the published FP32
# vector peak (157.3 TFLOP/s) without the factor 2 of the packed instructions;
# smf_measure_fma measures the rate on the device
VALU_FMA_PEAK = 256 * 4 * 16 * 2.4e9


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("rng.h", "device_path.h", "sample.hip", "rings.hip", "rings_fft.hip", "smf_internal.h"):
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


def time_split(plan, seed, count, out, steps, warmup):
    """Average ms per launch of the recursion and of the FFT inside one timed loop of the
    two launches of a sampling call (smf_sample_modes then smf_transform), HIP events
    between them on the launch stream."""
    import torch

    for _ in range(warmup):
        g = plan.sample_modes(seed, count, out)
        plan.transform(g, count)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for e in ev:
        e[0].record()
        g = plan.sample_modes(seed, count, out)
        e[1].record()
        plan.transform(g, count)
        e[2].record()
    torch.cuda.synchronize()
    rec = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    fft = sum(e[1].elapsed_time(e[2]) for e in ev) / steps
    return rec, fft


def alu_references(reps=5):
    """Throughput references measured on this device with the library's own kernels: the
    sampler's noise alone (Philox4x32-10 + FP32 Box-Muller, 8 blocks per stage in lockstep,
    no loads or stores) in normals/s, and unpacked FP32 FMAs in lane-FMAs/s; the best of
    `reps` timed launches after one warm-up each."""
    import ctypes

    import torch

    from paper_1709_10314_amd import smf

    lib = smf.load()
    st = torch.cuda.current_stream().cuda_stream
    wg = 256 * 4 * 8 // 4            # 8 waves per SIMD on 256 CUs, 4 waves per workgroup
    out = torch.empty(wg * 256, dtype=torch.float32, device="cuda")

    def best(launch):
        launch()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            rc = launch()
            e1.record()
            torch.cuda.synchronize()
            assert rc == 0, rc
            ts.append(e0.elapsed_time(e1))
        return min(ts)

    stages = 64
    ms_n = best(lambda: lib.smf_measure_normals(ctypes.c_uint64(1), wg, stages, ctypes.c_void_p(out.data_ptr()),
                                                ctypes.c_void_p(st)))
    normals = wg * 256 * stages * 32
    iters = 512
    ms_f = best(lambda: lib.smf_measure_fma(wg, iters, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st)))
    fmas = wg * 256 * iters * 128
    assert torch.isfinite(out).all()
    return {"normals_per_s": normals / (ms_n * 1e-3), "normals_ms": ms_n, "normals": normals,
            "fma_lane_per_s": fmas / (ms_f * 1e-3), "fma_ms": ms_f, "fmas": fmas,
            "fma_frac_of_unit_count_peak": fmas / (ms_f * 1e-3) / VALU_FMA_PEAK}


def markov_defect(cfg, modes=(0, 64, 1024, 3000), span=16):
    """The band-limit defect of reading 2 on the timed workload: for sampled modes, the
    chain's covariance between the start ring s and rings s-2 .. s-span (propagated through
    the oracle's factors) against J^m(z_s, z_r) of Lemma 2.1, relative to the geometric mean
    of the two variances; the largest over modes and rings."""
    import numpy as np

    import oracle
    from paper_1709_10314_amd import workloads

    n, order, lmax = cfg["n_theta"], cfg["order"], cfg["ell_max"]
    C = oracle.spectrum(workloads.kappas(cfg), lmax)
    s = oracle.start_ring(n)
    sets = span + 2
    A, B = oracle.setup_modes(order, C, n, list(modes), sets=sets)
    _, z = oracle.grid(n)
    worst = 0.0
    for k, m in enumerate(modes):
        S = B[0, k] @ B[0, k].T              # Cov(x_s, x_s)
        X = S.copy()                         # Cov(x_r, x_s), r walking north
        V = S.copy()
        for j in range(2, sets):
            r = s - j + 1
            X = A[j, k] @ X
            V = A[j, k] @ V @ A[j, k].T + B[j, k] @ B[j, k].T
            if s - r >= 2:
                J = oracle.jblock_z(order, m, lmax, C, z[r], z[s])
                worst = max(worst, abs(X[0, 0] - J[0, 0]) / np.sqrt(V[0, 0] * S[0, 0]))
    return {"max_rel_cov_defect": worst, "modes": list(modes), "rings": f"s-2 .. s-{span} against s"}


def batch_leg(steps, warmup):
    """The batched form on the 256-field mixed workload: one call samples every field after
    the launch-shape autotuner has run (m-tiles per chain item; two launches, or one
    persistent cooperative launch with a grid barrier between the chains and the rings); both
    forms are also timed at the chosen tile shape."""
    import torch

    from paper_1709_10314_amd import BatchPlan, workloads

    mix = workloads.batch_mix()
    fields = [dict(n_theta=w["n_theta"], n_phi=w["n_phi"], order=w["order"], kappa=[w["kappa"] ** 2] * w["order"],
                   ell_max=w["ell_max"]) for w in mix]
    t0 = time.perf_counter()
    bp = BatchPlan(fields)
    setup_s = time.perf_counter() - t0
    out = bp.empty()
    tiles = bp.autotune(1, out)
    _, persistent = bp.shape()
    ms, _ = time_calls(lambda: bp.sample(1, out), steps, warmup)
    forms = {}
    for p in (False, True):
        bp.set_shape(tiles, p)
        forms["ms_persistent" if p else "ms_two_launches"] = time_calls(lambda: bp.sample(1, out), steps, warmup)[0]
    bp.set_shape(tiles, persistent)
    pts = int(bp.offsets[-1])
    bp.close()
    del out
    torch.cuda.empty_cache()
    return {"value": pts / ms * 1e3, "unit": "grid points/s", "ms_per_step": ms, "fields": len(fields),
            "points": pts, "tiles": tiles, "persistent": persistent, **forms, "setup_s": setup_s,
            "workload": "256 fields: n_theta uniform on {128..2048}, n_phi = 2 n_theta, ln kappa ~ U(ln 2, ln 200), "
                        "order 1 or 2, FP32, seeds 1..256 (numpy PCG64(0))"}


def high_order_leg(cfg, order, steps, warmup, noise_peak):
    """The same grid and fields at Markov order 3 or 4 (C_l = (l(l+1) + kappa^2)^-M, FP32):
    ms per call, the recursion's ms per launch (events around smf_sample_modes) and its
    normals per second against the measured rate of the noise alone (noise_peak)."""
    import torch

    from paper_1709_10314_amd import Plan

    n, nphi, lmax, count, seed = cfg["n_theta"], cfg["n_phi"], cfg["ell_max"], cfg["count"], cfg["seed"]
    plan = Plan(order, n, nphi, lmax, kappa=[cfg["kappa"] ** 2] * order, precision="fp32")
    out = plan.empty(count)
    ms, _ = time_calls(lambda: plan.sample(seed, count, out), steps, warmup)
    ms_rec, _ = time_calls(lambda: plan.sample_modes(seed, count, out), steps, warmup)
    plan.close()
    del out
    torch.cuda.empty_cache()
    pts = count * n * nphi
    nps = pts * order / (ms_rec * 1e-3)
    return {"order": order, "value": pts / ms * 1e3, "unit": "grid points/s", "ms_per_step": ms,
            "recursion_ms": ms_rec, "normals_per_s": nps, "normals_frac_of_measured_noise_peak": nps / noise_peak}


def healpix_leg(steps, warmup, nside=1024, order=2, kappa=50.0, count=8, seed=1):
    """HEALPix rings (nside 1024: 4095 rings of 4k and 4 nside pixels, 12 nside^2 pixels per
    field) at ell_max = 3 nside - 1, order 2, FP32, 8 fields: ms per smf_sample_rings call
    (chains, then the ring synthesis) and per ring-synthesis launch, with the synthesis's
    algorithmic bytes (modes m <= m_top read once, pixels written once)."""
    import torch

    from paper_1709_10314_amd import RingPlan, workloads

    z, n_ring, phi0 = workloads.healpix_rings(nside)
    lmax = 3 * nside - 1
    t0 = time.perf_counter()
    plan = RingPlan(order, n_ring, phi0, lmax, kappa=[kappa ** 2] * order, precision="fp32", z=z)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    work = plan.empty(count)
    out = plan.empty_rings(count)
    ms, _ = time_calls(lambda: plan.sample_rings(seed, count, out, work), steps, warmup)
    plan.sample_modes(seed, count, work)
    ms_syn, _ = time_calls(lambda: plan.synthesize_rings(work, count, out), steps, warmup)
    pix = count * plan.pixels
    alg = count * (plan.n_theta * (plan.m_top + 1) * 8 + plan.pixels * 4)
    plan.close()
    del work, out
    torch.cuda.empty_cache()
    return {"workload": f"healpix-{nside}-M{order}-fp32-x{count}", "nside": nside, "rings": len(z),
            "pixels_per_field": int(n_ring.sum()), "ell_max": lmax, "order": order, "kappa": kappa,
            "fields": count, "value": pix / ms * 1e3, "unit": "pixels/s", "ms_per_step": ms,
            "synthesis_ms": ms_syn, "synthesis_alg_bytes": alg, "synthesis_alg_GBs": alg / (ms_syn * 1e-3) / 1e9,
            "synthesis_hbm_frac": alg / (ms_syn * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "synthesis_traffic": measured_traffic("ring_synthesis_healpix1024") if nside == 1024 and count == 8 else None,
            "setup_s": setup_s}


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(cfg, rings, single_rings):
    """The FP64 oracle (chains + naive DFT) on `rings` rings around the equator of every
    field of the workload, on all the threads the oracle uses; the same oracle on one
    thread for `single_rings` rings of field 1; and the oracle's chains followed by
    numpy's FFT in place of the naive DFT (a fair CPU speed for the sampling).  The factor
    sets the rings need are built first, untimed."""
    import numpy as np

    import oracle
    from paper_1709_10314_amd import workloads

    n, nphi, order, lmax, count = cfg["n_theta"], cfg["n_phi"], cfg["order"], cfg["ell_max"], cfg["count"]
    s = n // 2 - 1
    sets = rings // 2 + 1
    C = oracle.spectrum(workloads.kappas(cfg), lmax)
    t0 = time.perf_counter()
    A, B = oracle.setup(order, C, n, nphi, sets=sets)
    t_setup = time.perf_counter() - t0
    r0, r1 = s - rings // 2 + 1, s + rings // 2 + 1
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    g = oracle.sample_modes(order, n, A, B, cfg["seed"], count, sets=sets)
    T = oracle.dft(g, nphi, r0, r1)
    dt = time.perf_counter() - t0
    assert np.all(np.isfinite(T))
    pts = count * rings * nphi

    # one thread, a smaller sample: field 1, single_rings rings around the equator
    sets1 = single_rings // 2 + 1
    q0, q1 = s - single_rings // 2 + 1, s + single_rings // 2 + 1
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        g1 = oracle.sample_modes(order, n, A, B, cfg["seed"], 1, sets=sets1)
        T1 = oracle.dft(g1, nphi, q0, q1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    assert np.all(np.isfinite(T1))

    # chains + numpy irfft: T = g_0 + 2 sum Re(g_m e^{i m phi}) = n_phi * irfft(g)
    t0 = time.perf_counter()
    gf = oracle.sample_modes(order, n, A, B, cfg["seed"], count, sets=sets)
    X = np.zeros((count, rings, nphi // 2 + 1), dtype=np.complex128)
    X[:, :, : gf.shape[2]] = gf[:, r0:r1, :]
    X[:, :, 0] = X[:, :, 0].real
    Tf = np.fft.irfft(X, n=nphi, axis=-1) * nphi
    dtf = time.perf_counter() - t0
    err = float(np.max(np.abs(Tf - T)) / np.max(np.abs(T)))
    assert err < 1e-10, err
    return ({"value": pts / dt, "unit": "grid points/s", "cores": threads, "kind": "oracle",
            "sample": (f"{cfg['name']}: all {count} fields, the {rings} rings around the equator (all "
                       f"{lmax + 1} modes, {pts} points), chains + naive DFT in FP64; setup of the "
                       f"{sets} factor sets they need ({t_setup:.1f} s) not timed"),
            "seconds": dt, "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "single_thread": {"value": single_rings * nphi / dt1, "unit": "grid points/s", "cores": 1,
                              "sample": f"field 1, the {single_rings} rings around the equator", "seconds": dt1},
            "chains_plus_numpy_fft": {"value": pts / dtf, "unit": "grid points/s", "cores": threads,
                                      "sample": "same as the oracle sample; numpy.fft.irfft in place of the naive DFT",
                                      "seconds": dtf, "max_rel_diff_vs_oracle": err}}, T)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # untimed calls before the timed ones: about 30 calls (27 ms) bring the device to its
    # steady clocks (0.898 ms per step after 30 calls, 0.957 ms after 3, on the same box)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-high-order", action="store_true")
    ap.add_argument("--no-healpix", action="store_true")
    ap.add_argument("--cpu-rings", type=int, default=384)
    ap.add_argument("--cpu-single-rings", type=int, default=64)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (calibrates rocprofv3 FETCH/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the sampler shards by whole fields with no exchange between GPUs)",
              file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("RANK", "0")) != 0:
        return

    import numpy as np
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

    # the FP64 plain path first (the baseline of the FP32 path's speed-up, with the same
    # warm-up and half the timed steps); its calls also bring the device to its steady
    # clocks before the FP32 path is timed
    fp64 = None
    if not args.no_fp64:
        log("setup fp64 plain path")
        plan64 = Plan(order, n, nphi, lmax, kappa=workloads.kappas(cfg), precision="fp64")
        out64 = plan64.empty(count)
        ms64, _ = time_calls(lambda: plan64.sample(seed, count, out64), max(args.steps // 2, 3), args.warmup)
        plan64.close()
        del out64
        torch.cuda.empty_cache()
        fp64 = {"value": pts / ms64 * 1e3, "unit": "grid points/s", "ms_per_step": ms64,
                "warmup": args.warmup, "steps": max(args.steps // 2, 3)}
        log(f"  fp64 {ms64:.3f} ms/step")

    log(f"setup {cfg['name']} (fp32)")
    t0 = time.perf_counter()
    plan = Plan(order, n, nphi, lmax, kappa=workloads.kappas(cfg), precision="fp32")
    setup_s = time.perf_counter() - t0
    out = plan.empty(count)
    log(f"  setup {setup_s:.2f} s; timing {args.steps} steps")
    ms_step, wall_step = time_calls(lambda: plan.sample(seed, count, out), args.steps, args.warmup)
    log(f"  {ms_step:.3f} ms/step ({pts / ms_step * 1e3:.3e} pts/s)")
    ms_rec, ms_fft = time_split(plan, seed, count, out, args.steps, args.warmup)
    log(f"  recursion {ms_rec:.3f} ms, fft {ms_fft:.3f} ms per launch")
    m_top = plan.m_top
    n_sets = plan.n_sets
    # the timed output (its last call sampled seeds seed..seed+count-1): the rings around the
    # equator that the oracle sample of the cpu_baseline leg covers, kept for error_vs_oracle
    s_ring = n // 2 - 1
    r0, r1 = s_ring - args.cpu_rings // 2 + 1, s_ring + args.cpu_rings // 2 + 1
    torch.cuda.synchronize()
    T_gpu = out.view(count, n, nphi)[:, r0:r1, :].double().cpu().numpy()
    plan.close()
    del out
    torch.cuda.empty_cache()

    log("throughput references: Philox + Box-Muller alone, unpacked FP32 FMA")
    alu = alu_references()
    log(f"  {alu['normals_per_s']:.3e} normals/s, {alu['fma_lane_per_s']:.3e} lane-FMA/s "
        f"({100 * alu['fma_frac_of_unit_count_peak']:.0f}% of 256 x 4 x 16 x 2.4e9)")

    # algorithmic work per launch: the recursion reads the FP32 factors once and writes the
    # modes (and makes `order` normals per point); the FFT reads and writes every point once
    vals_per_rec = order * order + order * (order + 1) // 2
    fac_bytes = n_sets * (m_top + 1) * vals_per_rec * 4
    g_bytes = count * n * (nphi // 2) * 8
    kernels = {
        "recursion": {"ms": ms_rec, "alg_bytes": fac_bytes + g_bytes},
        "c2r_fft": {"ms": ms_fft, "alg_bytes": 2 * count * n * nphi * 4},
    }
    for k, v in kernels.items():
        v["alg_GBs"] = v["alg_bytes"] / (v["ms"] * 1e-3) / 1e9
        v["hbm_frac"] = v["alg_GBs"] / HBM_PEAK_GBS
    kr = kernels["recursion"]
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    kd = kernels[dom]
    traffic = measured_traffic(dom)
    if dom == "recursion":
        # ALU-bound: normals made per second against the generator's own measured rate
        nps = pts * order / (ms_rec * 1e-3)
        roofline = {"bound": "alu", "achieved": nps / 1e9, "peak": alu["normals_per_s"] / 1e9,
                    "unit": "G normals/s", "frac": nps / alu["normals_per_s"], "traffic": traffic,
                    "kernel": dom, "peak_source": "smf_measure_normals on this device"}
    else:
        roofline = {"bound": "hbm", "achieved": kd["alg_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": kd["hbm_frac"], "traffic": traffic, "kernel": dom}
    roofline["path_alg_GBs"] = (fac_bytes + g_bytes + 2 * count * n * nphi * 4) / (ms_step * 1e-3) / 1e9
    roofline["path_hbm_frac"] = roofline["path_alg_GBs"] / HBM_PEAK_GBS
    tr_fft = measured_traffic("c2r_fft")
    tr_rec = measured_traffic("recursion")
    if tr_fft is not None and tr_rec is not None:
        roofline["path_traffic_GBs"] = (tr_fft + tr_rec) / (ms_step * 1e-3) / 1e9
        roofline["path_traffic_frac"] = roofline["path_traffic_GBs"] / HBM_PEAK_GBS
    # normals per second of the recursion against the measured rate of the same generator
    # alone (smf_measure_normals: the noise with none of the recursion's loads and stores)
    kr["normals_per_s"] = pts * order / (ms_rec * 1e-3)
    kr["normals_frac_of_measured_noise_peak"] = kr["normals_per_s"] / alu["normals_per_s"]

    batch = None
    if not args.no_batch:
        log("batched form: 256-field mixed workload")
        batch = batch_leg(args.steps, args.warmup)
        log(f"  {batch['ms_per_step']:.3f} ms/call ({batch['value']:.3e} pts/s, tiles {batch['tiles']}, "
            f"setup {batch['setup_s']:.1f} s)")

    high = None
    if not args.no_high_order:
        high = []
        for o in (3, 4):
            log(f"order {o} on the same grid and fields")
            h = high_order_leg(cfg, o, args.steps, args.warmup, alu["normals_per_s"])
            log(f"  {h['ms_per_step']:.3f} ms/step, recursion {h['recursion_ms']:.3f} ms "
                f"({100 * h['normals_frac_of_measured_noise_peak']:.0f}% of the noise-alone rate)")
            high.append(h)

    hp = None
    if not args.no_healpix:
        log("HEALPix rings, nside 1024, order 2, 8 fields")
        hp = healpix_leg(args.steps, args.warmup)
        log(f"  {hp['ms_per_step']:.3f} ms/call ({hp['value']:.3e} pixels/s), ring synthesis "
            f"{hp['synthesis_ms']:.3f} ms ({hp['synthesis_alg_GBs']:.0f} GB/s algorithmic), setup {hp['setup_s']:.2f} s")

    cpu = None
    err = None
    defect = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on {args.cpu_rings} rings")
        cpu, T_orc = cpu_baseline(cfg, args.cpu_rings, args.cpu_single_rings)
        log(f"  {cpu['value']:.3e} pts/s on {cpu['cores']} threads in {cpu['seconds']:.1f} s")
        # the timed FP32 output against the FP64 oracle on the same normals, field by field
        d = T_gpu - T_orc
        rms = [float(np.sqrt(np.sum(d[f] ** 2) / np.sum(T_orc[f] ** 2))) for f in range(count)]
        mx = [float(np.max(np.abs(d[f])) / np.sqrt(np.mean(T_orc[f] ** 2))) for f in range(count)]
        err = {"per_field_rel_rms": rms, "per_field_max_abs_over_rms": mx, "bar_rel_rms": 1e-4,
               "fields": f"seeds {seed}..{seed + count - 1}", "rings": f"{r0}..{r1 - 1} of {n} (all modes, all phi)"}
        log(f"  timed output vs oracle: rel RMS up to {max(rms):.2e}, max |error| / RMS up to {max(mx):.2e}")
        log("markov defect of the band limit at sampled modes")
        defect = markov_defect(cfg)
        log(f"  {defect['max_rel_cov_defect']:.2e}")

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
        "batch_mix": batch,
        "higher_orders": high,
        "healpix": hp,
        "cpu_baseline": cpu,
        "error_vs_oracle": err,
        "markov_defect": defect,
        "alu_references": alu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
