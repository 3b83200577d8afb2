"""GPU parity of Markov orders 3 and 4 (state: the value and its first M-1 z-derivatives,
Sec. 2 Markov property; the higher derivatives from the associated Legendre equation)
against the FP64 oracle on the same Philox normals: factors by their action on the
chain's law (as for orders 1 and 2), modes and fields at the parity bars (FP64 1e-10, FP32
1e-4 relative RMS per field) for even and odd ring counts, truncated and band-limited
modes and an explicit grid; the layout rules (one part per lane, scans of at most 8 ring
blocks) and the batched form at every order.

At these orders the value and its derivatives are strongly correlated at a ring and the
factorisation is ill-conditioned: perturbing J by a few parts in 1e16 (FP64 rounding) moves
the sampled field by up to ~1e-7 at order 4 and ~1e-9 at order 3 (against ~1e-14 at order
2).  Two FP64 setups that sum J in different orders therefore agree only to that level, so
the checks are split:
  - the sampler, fed the oracle's own factors (smf_set_factors), against the oracle's
    samples at 1e-12 (FP64) and 1e-4 (FP32): the chain arithmetic and the noise alone;
  - the GPU setup against the oracle's, on the fields they produce, within a bound derived
    in the test from the oracle's own sensitivity: 20 times the field change that a random
    relative perturbation of J of 2.2e-16 causes (plus the 1e-10 bar), and the innovation
    covariances (factor_errors dB) within 1e-7."""
import numpy as np
import pytest

import oracle
from gpu_helpers import factor_errors, log, rel_rms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4}

# (order, kappa_i, n_theta, n_phi, ell_max)
CASES = [
    (3, 400.0, 64, 128, 63),
    (3, 2500.0, 33, 64, 40),
    (3, 50.0, 130, 256, 200),
    (4, 900.0, 32, 64, 31),
    (4, 100.0, 65, 128, 64),
    (4, 2500.0, 21, 256, 30),
]


def _plan(order, kap, n, nphi, lmax, precision, z=None):
    from paper_1709_10314_amd import Plan

    return Plan(order, n, nphi, lmax, kappa=[kap] * order, precision=precision, z=z)


def _perturbed_setup(order, C, n, nphi, lmax, rel, seed):
    """The oracle's factors with every J block perturbed by a random relative amount of
    size `rel` (symmetric for J(a,a), J(b,b)); the oracle's own factorisation."""
    import ctypes

    lib = oracle._load()
    lib.orc_step_factors.argtypes = [ctypes.c_int] + [ctypes.POINTER(ctypes.c_double)] * 5
    lib.orc_start_factor.argtypes = [ctypes.c_int] + [ctypes.POINTER(ctypes.c_double)] * 2

    def ptr(a):
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    rng = np.random.default_rng(seed)
    M = order
    mt, ns, s, even = oracle.m_top(lmax, nphi), oracle.n_sets(n), oracle.start_ring(n), n % 2 == 0
    A = np.zeros((ns, mt + 1, M, M))
    B = np.zeros((ns, mt + 1, M, M))

    def pert(K, sym):
        E = rng.standard_normal(K.shape)
        if sym:
            E = (E + E.T) / 2
        return np.ascontiguousarray(K * (1 + rel * E))

    for m in range(mt + 1):
        for j in range(ns):
            if j == 0:
                a = b = s
            elif even:
                a, b = (s, s + 1) if j == 1 else (s - j + 2, s - j + 1)
            else:
                a, b = s - j + 1, s - j
            Kaa = pert(oracle.jblock_ring(M, m, lmax, C, n, a, a), True)
            Bj = np.zeros(M * M)
            if j == 0:
                lib.orc_start_factor(M, ptr(Kaa), ptr(Bj))
                B[0, m] = Bj.reshape(M, M)
                continue
            Kbb = pert(oracle.jblock_ring(M, m, lmax, C, n, b, b), True)
            Kba = pert(oracle.jblock_ring(M, m, lmax, C, n, b, a), False)
            Aj = np.zeros(M * M)
            lib.orc_step_factors(M, ptr(Kaa), ptr(Kbb), ptr(Kba), ptr(Aj), ptr(Bj))
            A[j, m] = Aj.reshape(M, M)
            B[j, m] = Bj.reshape(M, M)
    return A, B


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "M%d-k%g-%dx%d-l%d" % c)
def test_high_order_sampler_on_oracle_factors(case, precision):
    """The chains and the FFT alone: the plan's factors replaced by the oracle's, modes and
    fields against the oracle's samples from the same factors and normals."""
    order, kap, n, nphi, lmax = case
    count, seed = 3, 31
    C = oracle.spectrum([kap] * order, lmax)
    A, B = oracle.setup(order, C, n, nphi)
    To, go = oracle.sample(order, n, nphi, A, B, seed, count)
    plan = _plan(order, kap, n, nphi, lmax, precision)
    plan.set_factors(A, B)
    Ag, Bg = plan.factors()
    assert np.array_equal(Ag[1:], A[1:]) and np.array_equal(np.tril(Bg), np.tril(B))
    mt = plan.m_top
    # the plain walk, then the affine scan (block transitions rebuilt from the given factors;
    # the fold adds the rounding of a product of up to ~n/2 transitions)
    bars = {("fp64", 1): 1e-12, ("fp64", 2): 1e-10, ("fp32", 1): 1e-4, ("fp32", 2): 1e-4}
    for blocks in (1, 4, 8):
        plan.set_ring_blocks(blocks)
        used = plan.ring_blocks(count)
        g = plan.sample_modes(seed, count)
        torch.cuda.synchronize()
        g = g.double().cpu().numpy()
        g = g[..., 0] + 1j * g[..., 1]
        T = plan.sample(seed, count)
        torch.cuda.synchronize()
        T = T.double().cpu().numpy()
        bar = bars[(precision, 1 if used == 1 else 2)]
        for f in range(count):
            eg = rel_rms(np.stack([g[f, :, : mt + 1].real, g[f, :, : mt + 1].imag]),
                         np.stack([go[f].real, go[f].imag]))
            eT = rel_rms(T[f], To[f])
            log(f"{case} {precision} on oracle factors, blocks {used}: field {f} modes {eg:.3e} field {eT:.3e}")
            assert eg <= bar and eT <= bar
    plan.close()


@pytest.mark.parametrize("case", CASES, ids=lambda c: "M%d-k%g-%dx%d-l%d" % c)
def test_high_order_setup_within_fp64_sensitivity(case):
    """The GPU setup against the oracle's on the fields they produce (FP64 sampling, same
    normals), within 20 times the change an FP64-sized perturbation of J causes in the
    oracle's own fields; the innovation covariances within 1e-7."""
    order, kap, n, nphi, lmax = case
    count, seed = 2, 31
    C = oracle.spectrum([kap] * order, lmax)
    Ao, Bo = oracle.setup(order, C, n, nphi)
    To, _ = oracle.sample(order, n, nphi, Ao, Bo, seed, count)
    Ap, Bp = _perturbed_setup(order, C, n, nphi, lmax, 2.2e-16, 7)
    Tp, _ = oracle.sample(order, n, nphi, Ap, Bp, seed, count)
    sens = max(rel_rms(Tp[f], To[f]) for f in range(count))
    plan = _plan(order, kap, n, nphi, lmax, "fp64")
    Ag, Bg = plan.factors()
    T = plan.sample(seed, count)
    torch.cuda.synchronize()
    T = T.cpu().numpy()
    plan.close()
    e = max(rel_rms(T[f], To[f]) for f in range(count))
    _, dB, amb = factor_errors(Ag, Bg, Ao, Bo, n)
    bound = 1e-10 + 20 * sens
    log(f"{case}: GPU setup field vs oracle {e:.3e}; oracle's own FP64 sensitivity {sens:.3e} "
        f"(bound {bound:.3e}); dB {dB:.3e} ({amb} steps next to a threshold)")
    assert e <= bound
    assert dB < 1e-7


@pytest.mark.parametrize("case", CASES, ids=lambda c: "M%d-k%g-%dx%d-l%d" % c)
def test_high_order_fp32_modes_and_field_match_oracle(case):
    """The FP32 path end to end (GPU setup, FP32 sampling) against the oracle at 1e-4."""
    precision = "fp32"
    order, kap, n, nphi, lmax = case
    count, seed = 3, 31
    plan = _plan(order, kap, n, nphi, lmax, precision)
    log(f"{case} {precision}: ring blocks {plan.ring_blocks(count)}")
    g = plan.sample_modes(seed, count)
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    g = g[..., 0] + 1j * g[..., 1]
    T = plan.sample(seed, count)
    torch.cuda.synchronize()
    T = T.double().cpu().numpy()
    mt = plan.m_top
    plan.close()
    C = oracle.spectrum([kap] * order, lmax)
    A, B = oracle.setup(order, C, n, nphi)
    To, go = oracle.sample(order, n, nphi, A, B, seed, count)
    assert np.all(g[:, :, mt + 1:] == 0)
    for f in range(count):
        eg = rel_rms(np.stack([g[f, :, : mt + 1].real, g[f, :, : mt + 1].imag]),
                     np.stack([go[f].real, go[f].imag]))
        eT = rel_rms(T[f], To[f])
        log(f"{case} {precision}: field {f} modes {eg:.3e} field {eT:.3e}")
        assert eg <= TOL[precision] and eT <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_order3_on_gauss_legendre_grid(precision):
    """Order 3 on an explicit grid, end to end (this case is well conditioned: its FP64
    fields agree at the 1e-10 bar)."""
    from paper_1709_10314_amd import workloads

    z = workloads.gauss_legendre_z(48)
    order, kap, nphi, lmax = 3, 900.0, 64, 47
    plan = _plan(order, kap, len(z), nphi, lmax, precision, z=z)
    T = plan.sample(5, 2)
    torch.cuda.synchronize()
    T = T.double().cpu().numpy()
    plan.close()
    C = oracle.spectrum([kap] * order, lmax)
    A, B = oracle.setup(order, C, len(z), nphi, z=z)
    To, _ = oracle.sample(order, len(z), nphi, A, B, 5, 2)
    e = max(rel_rms(T[f], To[f]) for f in range(2))
    log(f"order 3 on Gauss-Legendre 48 {precision}: {e:.3e}")
    assert e <= TOL[precision]


def test_high_order_layout_and_limits():
    """Orders 3 and 4 run one part per lane; the automatic layout scans with the fewest
    blocks (at most 8) giving 4096 waves below 1024 waves of plain recursion, and plain
    above; forced layouts cap at 8 blocks; a field's result depends on the blocks only
    (the same field in a 1-field and a 32-field call with 8 blocks is bit identical)."""
    plan = _plan(3, 400.0, 1024, 2048, 1023, "fp32")
    assert [plan.ring_blocks(c) for c in (1, 8, 16, 64)] == [8, 8, 1, 1]
    plan.set_ring_blocks(16)
    assert [plan.ring_blocks(c) for c in (1, 64)] == [8, 8]
    plan.set_ring_blocks(8)
    a = plan.sample(7, 1)[0].clone()
    b = plan.sample(7, 32)[0]
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.set_ring_blocks(1)
    c = plan.sample(7, 1)[0]
    torch.cuda.synchronize()
    e = rel_rms(c.double().cpu().numpy(), a.double().cpu().numpy())
    log(f"1024x2048 M3 fp32: 8-block scan vs plain {e:.3e}")
    assert e <= 2e-5
    plan.close()


@pytest.mark.parametrize("order", [3, 4])
def test_high_order_chains_per_lane_do_not_change_results(order):
    """The plain recursion with two parts per lane (a 64-field call, 4096 one-part waves) and
    with one (a 16-field call) give field 0 bit for bit."""
    plan = _plan(order, 400.0, 1024, 2048, 1023, "fp32")
    plan.set_ring_blocks(1)
    a = plan.sample(9, 16)[0].clone()
    b = plan.sample(9, 64)[0]
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.close()


def test_batch_with_orders_1_to_4():
    """The batched form on fields of every order: each field against the same field sampled
    alone with the plain recursion (the same chain arithmetic) and against the oracle."""
    from paper_1709_10314_amd import BatchPlan

    fields = [dict(n_theta=64, n_phi=128, order=3, kappa=[400.0] * 3, ell_max=63),
              dict(n_theta=33, n_phi=64, order=4, kappa=[900.0] * 4, ell_max=31),
              dict(n_theta=130, n_phi=256, order=2, kappa=[700.0] * 2, ell_max=129),
              dict(n_theta=65, n_phi=128, order=1, kappa=[100.0], ell_max=64),
              dict(n_theta=256, n_phi=512, order=3, kappa=[50.0] * 3, ell_max=255)]
    seed = 11
    bp = BatchPlan(fields)
    out = bp.sample(seed)
    torch.cuda.synchronize()
    for i, f in enumerate(fields):
        Tb = bp.field(out, i).double().cpu().numpy()
        plan = _plan(f["order"], f["kappa"][0], f["n_theta"], f["n_phi"], f["ell_max"], "fp32")
        plan.set_ring_blocks(1)
        Ts = plan.sample(seed + i, 1)[0]
        torch.cuda.synchronize()
        Ts = Ts.double().cpu().numpy()
        plan.close()
        C = oracle.spectrum(f["kappa"], f["ell_max"])
        A, B = oracle.setup(f["order"], C, f["n_theta"], f["n_phi"])
        To, _ = oracle.sample(f["order"], f["n_theta"], f["n_phi"], A, B, seed + i, 1)
        es, eo = rel_rms(Tb, Ts), rel_rms(Tb, To[0])
        log(f"batch field {i} (order {f['order']}): vs single plan {es:.2e}, vs oracle {eo:.2e}")
        assert es <= 1e-6 and eo <= TOL["fp32"]
    bp.close()


def test_order3_large_single_field_modes():
    """One 1024 x 2048 order-3 field in FP32 (the automatic layout scans it with 8 blocks):
    sampled modes against the oracle's chains of those modes."""
    n, nphi, lmax, kap = 1024, 2048, 1023, 2500.0
    plan = _plan(3, kap, n, nphi, lmax, "fp32")
    g = plan.sample_modes(3, 2)
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    g = g[..., 0] + 1j * g[..., 1]
    plan.close()
    ms = [0, 1, 5, 100, 511, 1000, 1023]
    C = oracle.spectrum([kap] * 3, lmax)
    A, B = oracle.setup_modes(3, C, n, ms)
    go = oracle.sample_modes_list(3, n, ms, A, B, 3, 2)
    for f in range(2):
        e = rel_rms(np.stack([g[f][:, ms].real, g[f][:, ms].imag]), np.stack([go[f].real, go[f].imag]))
        log(f"1024x2048 M3 fp32 field {f}: sampled modes vs oracle {e:.3e}")
        assert e <= TOL["fp32"]


@pytest.mark.parametrize("blocks", [1, 4])
def test_order3_on_a_grid_with_no_symmetry(blocks):
    """Order 3 on shifted ring centres: the plan's 2 n_sets factor sets replaced by the
    oracle's (northern, then the southern walk's in true coordinates), plain and scanned,
    against the oracle's sampler with its southern sets (FP64, chain arithmetic only)."""
    from paper_1709_10314_amd import workloads

    z = workloads.shifted_z(48, 0.3)
    kap, nphi, lmax = 900.0, 64, 47
    C = oracle.spectrum([kap] * 3, lmax)
    A, B, As, Bs = oracle.setup_asym(3, C, len(z), nphi, z)
    To, _ = oracle.sample(3, len(z), nphi, A, B, 4, 2, south=(As, Bs))
    plan = _plan(3, kap, len(z), nphi, lmax, "fp64", z=z)
    assert not plan.symmetric
    plan.set_factors(np.concatenate([A, As]), np.concatenate([B, Bs]))
    plan.set_ring_blocks(blocks)
    T = plan.sample(4, 2)
    torch.cuda.synchronize()
    T = T.cpu().numpy()
    used = plan.ring_blocks(2)
    plan.close()
    e = max(rel_rms(T[f], To[f]) for f in range(2))
    log(f"order 3, shifted grid, blocks {used}: {e:.3e}")
    assert e <= 1e-10
