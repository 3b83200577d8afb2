"""GPU parity of the affine scan across ring blocks (the chains cut into blocks that run in
parallel and are joined through the block transitions): modes and fields against the FP64
oracle at the same bars as the plain recursion (FP64 1e-10, FP32 1e-4 relative RMS), for
both orders, odd and even ring counts, truncated and band-limited modes and every block
count; the scan against the plain recursion of the same plan (rounding only); the
automatic choice of the block count; and argument checks."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_rms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4}
# the scan and the plain recursion of one plan differ by the rounding of the block
# transitions and of the fold (a few hundred roundings of the working precision)
SAME = {"fp64": 1e-12, "fp32": 2e-5}

# (order, kappa_i, n_theta, n_phi, ell_max): walks of 31..255 main steps (fine blocks 2..16)
CASES = [
    (1, 64.0, 64, 128, 63),
    (2, 2500.0, 64, 128, 63),
    (2, 100.0, 67, 128, 50),
    (1, 400.0, 129, 64, 40),
    (2, 700.0, 130, 256, 200),
    (1, 30.0, 255, 512, 254),
    (2, 900.0, 512, 256, 511),
]


def _plan(order, kappa, n_theta, n_phi, ell_max, precision):
    from paper_1709_10314_amd import Plan

    return Plan(order, n_theta, n_phi, ell_max, kappa=[kappa] * order, precision=precision)


def _run(plan, blocks, seed, count):
    plan.set_ring_blocks(blocks)
    g = plan.sample_modes(seed, count)
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    T = plan.sample(seed, count)
    torch.cuda.synchronize()
    return g[..., 0] + 1j * g[..., 1], T.double().cpu().numpy()


def _fine(n_theta):
    walk = (n_theta // 2 + 1 - 2) if n_theta % 2 == 0 else ((n_theta + 1) // 2 - 1)
    b = 1
    while b < 16 and walk // (2 * b) >= 8:
        b *= 2
    return b


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "M%d-k%g-%dx%d-l%d" % c)
def test_scan_matches_oracle_and_plain(case, precision):
    order, kap, n, nphi, lmax = case
    count, seed = 2, 23
    plan = _plan(order, kap, n, nphi, lmax, precision)
    mt = plan.m_top
    g1, T1 = _run(plan, 1, seed, count)
    assert plan.ring_blocks(count) == 1
    C = oracle.spectrum([kap] * order, lmax)
    A, B = oracle.setup(order, C, n, nphi)
    To, go = oracle.sample(order, n, nphi, A, B, seed, count)
    fine = _fine(n)
    for blocks in (2, 4, 8, 16):
        g, T = _run(plan, blocks, seed, count)
        used = plan.ring_blocks(count)
        assert used == min(blocks, fine, 8 if precision == "fp64" else 16)
        assert np.all(g[:, :, mt + 1:] == 0)
        for f in range(count):
            eg = rel_rms(np.stack([g[f, :, : mt + 1].real, g[f, :, : mt + 1].imag]),
                         np.stack([go[f].real, go[f].imag]))
            eT = rel_rms(T[f], To[f])
            es = rel_rms(T[f], T1[f])
            log(f"{case} {precision} blocks {used}: field {f} modes {eg:.2e} field {eT:.2e} vs plain {es:.2e}")
            assert eg <= TOL[precision] and eT <= TOL[precision]
            assert es <= SAME[precision]
    plan.close()


def test_single_large_field_scans_and_matches_oracle_modes():
    """One 4096 x 8192 order-2 field: the automatic rule cuts its 16,382 chains into 16
    blocks; sampled modes against the oracle chains, and the field against the plain
    recursion of the same plan."""
    n, nphi, lmax, kap = 4096, 8192, 4095, 2500.0
    plan = _plan(2, kap, n, nphi, lmax, "fp32")
    assert plan.ring_blocks(1) == 16
    assert plan.ring_blocks(8) == 1
    plan.set_ring_blocks(0)
    g = plan.sample_modes(3, 1)
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    g = g[..., 0] + 1j * g[..., 1]
    T = plan.sample(3, 1).clone()
    plan.set_ring_blocks(1)
    T1 = plan.sample(3, 1)
    torch.cuda.synchronize()
    es = rel_rms(T.double().cpu().numpy(), T1.double().cpu().numpy())
    log(f"4096x8192 x1: scan vs plain field {es:.2e}")
    assert es <= SAME["fp32"]
    plan.close()
    ms = [0, 1, 7, 300, 2047, 4000, 4095]
    C = oracle.spectrum([kap, kap], lmax)
    A, B = oracle.setup_modes(2, C, n, ms)
    go = oracle.sample_modes_list(2, n, ms, A, B, 3, 1)
    e = rel_rms(np.stack([g[0][:, ms].real, g[0][:, ms].imag]), np.stack([go[0].real, go[0].imag]))
    log(f"4096x8192 x1: sampled modes vs oracle {e:.2e}")
    assert e <= TOL["fp32"]


def test_scan_modes_are_deterministic():
    plan = _plan(2, 100.0, 256, 512, 255, "fp32")
    plan.set_ring_blocks(8)
    a = plan.sample(5, 2).clone()
    b = plan.sample(5, 2)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.close()


def test_ring_blocks_arguments():
    from paper_1709_10314_amd import SmfError, smf

    plan = _plan(1, 30.0, 64, 128, 63, "fp64")
    for bad in (-1, 3, 6, 17, 32):
        with pytest.raises(SmfError):
            plan.set_ring_blocks(bad)
    rc, _ = smf.smf_get_ring_blocks(plan.handle, -1)
    assert rc == smf.SMF_EINVAL
    assert plan.ring_blocks(1) == 1          # automatic: 31 main steps are too short to cut
    plan.set_ring_blocks(16)
    assert plan.ring_blocks(1) == 2          # forced: at most 2 blocks of >= 8 steps
    plan.close()
    mid = _plan(2, 400.0, 1024, 2048, 1023, "fp64")
    assert [mid.ring_blocks(c) for c in (1, 4, 8, 15, 16)] == [8, 8, 8, 8, 1]
    mid.close()
    tiny = _plan(2, 9.0, 16, 32, 15, "fp64")   # 7 main steps: no scan
    tiny.set_ring_blocks(4)
    assert tiny.ring_blocks(1) == 1
    tiny.close()


def test_chains_per_lane_do_not_change_results():
    """The per-call layout (one or two chains per lane) is a performance choice only: field 0
    of a 1-field call and of a 32-field call (one-part and two-part plain recursion) are bit
    identical, and so are forced 8-block scans of a 1-field and an 8-field call (one-part and
    two-part scan)."""
    plan = _plan(2, 400.0, 1024, 2048, 1023, "fp32")
    plan.set_ring_blocks(1)
    a = plan.sample(9, 1)[0].clone()
    b = plan.sample(9, 32)[0].clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.set_ring_blocks(8)
    assert plan.ring_blocks(1) == 8 and plan.ring_blocks(8) == 8
    c = plan.sample(9, 1)[0].clone()
    d = plan.sample(9, 8)[0].clone()
    torch.cuda.synchronize()
    assert torch.equal(c, d)
    e = rel_rms(c.double().cpu().numpy(), a.double().cpu().numpy())
    log(f"1024x2048 M2 fp32: 8-block scan vs plain {e:.2e}")
    assert e <= SAME["fp32"]
    plan.close()


def test_two_part_scan_matches_oracle_modes():
    """8 fields of 1024 x 2048, order 2, FP32: the automatic choice is an 8-block scan with
    two chains per lane; sampled modes of two fields against the oracle."""
    n, nphi, lmax, kap = 1024, 2048, 1023, 400.0
    plan = _plan(2, kap, n, nphi, lmax, "fp32")
    assert plan.ring_blocks(8) == 8
    g = plan.sample_modes(21, 8)
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    g = g[..., 0] + 1j * g[..., 1]
    plan.close()
    ms = [0, 1, 2, 100, 511, 1000, 1023]
    C = oracle.spectrum([kap, kap], lmax)
    A, B = oracle.setup_modes(2, C, n, ms)
    go = oracle.sample_modes_list(2, n, ms, A, B, 21, 8)
    for f in (0, 7):
        e = rel_rms(np.stack([g[f][:, ms].real, g[f][:, ms].imag]), np.stack([go[f].real, go[f].imag]))
        log(f"1024x2048 x8 two-part scan: field {f} sampled modes vs oracle {e:.2e}")
        assert e <= TOL["fp32"]


@pytest.mark.parametrize("blocks", [1, 8])
def test_single_plan_graph_capture_replays(blocks):
    """smf_sample (plain recursion or scan, then the FFT) captured in a HIP graph: every
    replay, with eager work and synchronisations between replays, equals the eager call."""
    plan = _plan(2, 900.0, 512, 1024, 511, "fp32")
    plan.set_ring_blocks(blocks)
    eager = plan.sample(13, 2).clone()
    torch.cuda.synchronize()
    out = plan.empty(2)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.sample(13, 2, out, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.sample(13, 2, out, stream=s)
    for rep in range(3):
        out.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), (blocks, rep)
        del junk
    plan.close()
