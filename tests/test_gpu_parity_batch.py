"""GPU tests of the batched form: every field of a mixed batch against the same field
sampled alone (same device arithmetic, so equal to FP32 rounding) and against the FP64
oracle (1e-4), HIP-graph capture and replay, and the tile-shape autotuner."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_rms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mixed_fields():
    """Small uneven batch: odd/even rings, both orders, truncated and band-limited modes."""
    out = []
    specs = [(8, 16, 1, 30.0, 7), (33, 64, 2, 5.0, 31), (64, 128, 1, 400.0, 63), (16, 32, 2, 2500.0, 15),
             (128, 256, 2, 90.0, 127), (21, 64, 1, 3.0, 40), (2, 4, 2, 10.0, 3), (256, 512, 1, 1e4, 255),
             (100, 128, 2, 700.0, 80), (64, 4096, 1, 16.0, 63), (512, 1024, 2, 2500.0, 511)]
    for n, nphi, order, kap, lmax in specs:
        out.append(dict(n_theta=n, n_phi=nphi, order=order, kappa=[kap] * order, ell_max=lmax))
    return out


def _single(f, seed):
    from paper_1709_10314_amd import Plan

    p = Plan(f["order"], f["n_theta"], f["n_phi"], f["ell_max"], kappa=f["kappa"], precision="fp32")
    T = p.sample(seed, 1)
    torch.cuda.synchronize()
    T = T[0].double().cpu().numpy()
    p.close()
    return T


def test_batch_matches_single_plans_and_oracle():
    from paper_1709_10314_amd import BatchPlan

    fields = _mixed_fields()
    bp = BatchPlan(fields)
    out = bp.sample(40)
    for i, f in enumerate(fields):
        Tb = bp.field(out, i).double().cpu().numpy()
        Ts = _single(f, 40 + i)
        e1 = rel_rms(Tb, Ts)
        C = oracle.spectrum(f["kappa"], f["ell_max"])
        A, B = oracle.setup(f["order"], C, f["n_theta"], f["n_phi"])
        To, _ = oracle.sample(f["order"], f["n_theta"], f["n_phi"], A, B, 40 + i, 1)
        e2 = rel_rms(Tb, To[0])
        log(f"field {i} {f['n_theta']}x{f['n_phi']} M{f['order']}: vs single {e1:.2e}, vs oracle {e2:.2e}")
        assert e1 <= 1e-6 and e2 <= 1e-4
    bp.close()


def test_batch_graph_capture_replays():
    """One graph holds both launches; every replay, with eager work and synchronisations
    between replays, equals the eager result."""
    from paper_1709_10314_amd import BatchPlan

    fields = _mixed_fields()[:6]
    bp = BatchPlan(fields)
    eager = bp.sample(7).clone()
    torch.cuda.synchronize()
    out = bp.empty()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        bp.sample(7, out, stream=s)          # warm-up on the capture stream
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        bp.sample(7, out, stream=s)
    for rep in range(3):
        out.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        del junk
    bp.close()


def test_batch_autotune_keeps_results():
    from paper_1709_10314_amd import BatchPlan

    fields = _mixed_fields()
    bp = BatchPlan(fields)
    ref = bp.sample(3).clone()
    out = bp.empty()
    tiles = bp.autotune(3, out)
    log(f"autotuned m-tiles per chain item: {tiles}")
    assert tiles in (1, 2, 4)
    out2 = bp.sample(3)
    torch.cuda.synchronize()
    assert torch.equal(out2, ref)
    bp.close()


def test_batch_rejects_bad_arguments():
    from paper_1709_10314_amd import smf

    f = dict(n_theta=8, n_phi=16, order=1, kappa=[4.0], ell_max=7)
    rc, _ = smf.smf_setup_batch([f], flags=smf.SMF_FP64)
    assert rc == smf.SMF_EINVAL
    rc, _ = smf.smf_setup_batch([dict(f, n_phi=8192)])
    assert rc == smf.SMF_EINVAL
    rc, _ = smf.smf_setup_batch([f, dict(f, kappa=[0.0])])
    assert rc == smf.SMF_ENUMERIC
    from paper_1709_10314_amd import BatchPlan

    bp = BatchPlan([f])
    assert smf.smf_sample(bp.handle, 1, 1, 0) == smf.SMF_EINVAL     # not a single-field plan
    bp.close()


def test_mixed_256_field_workload_sampled():
    """The 256-field mixed workload (n_theta in {128..2048}, n_phi = 2 n_theta, kappa
    log-uniform in [2, 200], order 1 or 2): eight fields compared with their single-plan
    samples, two with the oracle."""
    from paper_1709_10314_amd import BatchPlan, workloads

    mix = workloads.batch_mix()
    fields = [dict(n_theta=w["n_theta"], n_phi=w["n_phi"], order=w["order"],
                   kappa=[w["kappa"] ** 2] * w["order"], ell_max=w["ell_max"]) for w in mix]
    log("setup 256 fields")
    bp = BatchPlan(fields)
    out = bp.sample(1)
    pts = bp.offsets[-1]
    log(f"{pts} points")
    for i in (0, 1, 17, 64, 128, 200, 254, 255):
        Tb = bp.field(out, i).double().cpu().numpy()
        Ts = _single(fields[i], 1 + i)
        e = rel_rms(Tb, Ts)
        log(f"field {i} {fields[i]['n_theta']} M{fields[i]['order']}: vs single {e:.2e}")
        assert e <= 1e-6
    small = [i for i, f in enumerate(fields) if f["n_theta"] == 128][:2]
    for i in small:
        f = fields[i]
        C = oracle.spectrum(f["kappa"], f["ell_max"])
        A, B = oracle.setup(f["order"], C, f["n_theta"], f["n_phi"])
        To, _ = oracle.sample(f["order"], f["n_theta"], f["n_phi"], A, B, 1 + i, 1)
        e = rel_rms(bp.field(out, i).double().cpu().numpy(), To[0])
        log(f"field {i}: vs oracle {e:.2e}")
        assert e <= 1e-4
    bp.close()
