"""GPU tests of the batched form: every field of a mixed batch against the same field
sampled alone (same device arithmetic, so equal to FP32 rounding) and against the FP64
oracle (1e-4), HIP-graph capture and replay, the persistent form (one cooperative launch)
against the two-launch form, and the launch-shape autotuner."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, max_rel_err, rel_rms

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
    log(f"autotuned launch shape: {bp.shape()}")
    assert tiles in (1, 2, 4) and bp.shape()[0] == tiles
    out2 = bp.sample(3)
    torch.cuda.synchronize()
    worst = max(max_rel_err(bp.field(out2, i).double().cpu().numpy(), bp.field(ref, i).double().cpu().numpy())
                for i in range(len(fields)))
    assert worst <= 2e-6     # FP32 rounding: the shapes' ring transforms may contract differently
    bp.close()


@pytest.mark.parametrize("tiles", [1, 2, 4])
def test_batch_persistent_form_equals_two_launches(tiles):
    """One cooperative launch (chain items, grid barrier, ring items) gives the two-launch
    result, in both the packed and the per-field form: bit for bit where its ring phase runs
    the same 256 threads per row (2 m-tiles), else to FP32 rounding (the transform compiled for
    128 or 512 threads may contract its multiply-adds differently)."""
    from paper_1709_10314_amd import BatchPlan

    fields = _mixed_fields()
    bp = BatchPlan(fields)
    bp.set_shape(2, False)
    ref = bp.sample(21).clone()
    outs_ref = [o.clone() for o in bp.sample_fields([5 + 3 * i for i in range(len(fields))])]
    torch.cuda.synchronize()
    bp.set_shape(tiles, True)
    assert bp.shape() == (tiles, True)
    out = bp.sample(21)
    outs = bp.sample_fields([5 + 3 * i for i in range(len(fields))])
    torch.cuda.synchronize()
    if tiles == 2:
        assert torch.equal(out, ref)
        for a, b in zip(outs, outs_ref):
            assert torch.equal(a, b)
    worst = 0.0
    for i in range(len(fields)):
        worst = max(worst, max_rel_err(bp.field(out, i).double().cpu().numpy(), bp.field(ref, i).double().cpu().numpy()),
                    max_rel_err(outs[i].double().cpu().numpy(), outs_ref[i].double().cpu().numpy()))
    log(f"persistent form, {tiles} m-tiles: largest element difference {worst:.2e} of the field RMS")
    assert worst <= 2e-6
    bp.close()


def test_batch_persistent_graph_capture_replays():
    """The persistent form captured in a HIP graph: every replay, with eager work and
    synchronisations between replays, equals the eager two-launch result."""
    from paper_1709_10314_amd import BatchPlan

    fields = _mixed_fields()[:6]
    bp = BatchPlan(fields)
    eager = bp.sample(7).clone()
    torch.cuda.synchronize()
    bp.set_shape(2, True)
    out = bp.empty()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        bp.sample(7, out, stream=s)
    torch.cuda.synchronize()
    assert torch.equal(out, eager)
    with torch.cuda.graph(g, stream=s):
        bp.sample(7, out, stream=s)
    for rep in range(3):
        out.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        del junk
    bp.close()


def test_batch_shape_arguments():
    from paper_1709_10314_amd import BatchPlan, smf

    bp = BatchPlan(_mixed_fields()[:2])
    for t, p in ((3, 0), (0, 1), (2, 2), (8, 0)):
        assert smf.load().smf_batch_set_shape(bp.handle, t, p) == smf.SMF_EINVAL
    assert bp.shape() == (2, False)
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
        Tb = bp.field(out, i).double().cpu().numpy()
        e, emax = rel_rms(Tb, To[0]), max_rel_err(Tb, To[0])
        log(f"field {i}: vs oracle {e:.2e} (max {emax:.2e})")
        assert e <= 1e-4 and emax <= 1e-3
    # one field of each ring count against the oracle: the rings around the equator (every
    # mode, from the factor sets near the start) and sampled modes over every ring (the
    # modes of the output recovered by a forward real FFT of each ring, g_m = rfft(T)_m / n_phi)
    for n in (128, 256, 512, 1024, 2048):
        i = next(k for k, f in enumerate(fields) if f["n_theta"] == n)
        f = fields[i]
        Tb = bp.field(out, i).double().cpu().numpy()
        e_r, e_m = _oracle_rings_and_modes(f, 1 + i, Tb)
        log(f"field {i} {n}x{f['n_phi']} M{f['order']}: equator rings vs oracle {e_r:.2e}, "
            f"modes vs oracle {max(e_m):.2e}")
        assert e_r <= 1e-4 and max(e_m) <= 1e-4
    bp.close()


def _oracle_rings_and_modes(f, seed, T, sets=9, modes=(0, 1, 5, 33)):
    """Relative RMS error of the rings reached by the first `sets` factor sets (around the
    equator) and of the listed modes over every ring, against the oracle."""
    n, nphi, order = f["n_theta"], f["n_phi"], f["order"]
    C = oracle.spectrum(f["kappa"], f["ell_max"])
    s = oracle.start_ring(n)
    A, B = oracle.setup(order, C, n, nphi, sets=sets)
    g = oracle.sample_modes(order, n, A, B, seed, 1, sets=sets)
    r0, r1 = s - sets + 2, s + sets
    To = oracle.dft(g, nphi, r0, r1)[0]
    e_r = rel_rms(T[r0:r1], To)
    md = [m for m in modes if m <= oracle.m_top(f["ell_max"], nphi)]
    Am, Bm = oracle.setup_modes(order, C, n, md)
    go = oracle.sample_modes_list(order, n, md, Am, Bm, seed, 1)[0]
    G = np.fft.rfft(T, axis=1) / nphi
    e_m = []
    for k, m in enumerate(md):
        a = np.stack([G[:, m].real, G[:, m].imag])
        b = np.stack([go[:, k].real, go[:, k].imag])
        e_m.append(rel_rms(a, b))
    return e_r, e_m


def test_batch_per_field_buffers_and_seeds():
    """smf_sample_batch with one seed and one device buffer per field: with seeds seed + i it
    equals the packed form field by field; with arbitrary seeds each field equals its single
    plan with that seed and the oracle; calls on two streams in a row, each with its own
    buffers, keep their own seeds."""
    from paper_1709_10314_amd import BatchPlan

    fields = _mixed_fields()
    bp = BatchPlan(fields)
    packed = bp.sample(40)
    outs = bp.sample_fields([40 + i for i in range(bp.n)])
    torch.cuda.synchronize()
    for i in range(bp.n):
        assert torch.equal(outs[i].view(-1), bp.field(packed, i).reshape(-1)), i
    seeds = [1000 + 7 * i * i for i in range(bp.n)]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(s1):
        o1 = bp.sample_fields(seeds, stream=s1)
    with torch.cuda.stream(s2):
        o2 = bp.sample_fields([x + 1 for x in seeds], stream=s2)
    torch.cuda.synchronize()
    for i, f in enumerate(fields):
        Ts = _single(f, seeds[i])
        e1 = rel_rms(o1[i].double().cpu().numpy(), Ts)
        e2 = rel_rms(o2[i].double().cpu().numpy(), _single(f, seeds[i] + 1))
        log(f"field {i}: per-field buffers vs single plan {e1:.2e} / {e2:.2e}")
        assert e1 <= 1e-6 and e2 <= 1e-6
    for i in (0, 3, 10):
        f = fields[i]
        C = oracle.spectrum(f["kappa"], f["ell_max"])
        A, B = oracle.setup(f["order"], C, f["n_theta"], f["n_phi"])
        To, _ = oracle.sample(f["order"], f["n_theta"], f["n_phi"], A, B, seeds[i], 1)
        e = rel_rms(o1[i].double().cpu().numpy(), To[0])
        log(f"field {i}: per-field buffers vs oracle {e:.2e}")
        assert e <= 1e-4
    bp.close()


def test_batch_per_field_rejects_bad_buffers():
    from paper_1709_10314_amd import BatchPlan, smf

    f = dict(n_theta=8, n_phi=16, order=1, kappa=[4.0], ell_max=7)
    bp = BatchPlan([f, f])
    a = torch.empty(128, device="cuda")
    assert smf.smf_sample_batch(bp.handle, [1, 2], [a.data_ptr(), 0]) == smf.SMF_EINVAL
    assert smf.smf_sample_batch(bp.handle, [1, 2], [a.data_ptr(), a.data_ptr() + 4]) == smf.SMF_EINVAL
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    b = torch.empty(128, device="cuda")
    with torch.cuda.graph(g, stream=s):
        b.zero_()
        rc = smf.smf_sample_batch(bp.handle, [1, 2], [a.data_ptr(), b.data_ptr()], stream=s)
    assert rc == smf.SMF_EINVAL          # capturing: the packed form is the capturable one
    bp.close()
