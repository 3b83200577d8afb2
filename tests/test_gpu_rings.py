"""GPU parity on rings with their own pixel counts and first-pixel longitudes (iso-latitude
grids such as HEALPix, Sec. 1; Alg. 2's last step evaluated at each ring's pixels with every
mode kept): the ring synthesis alone on seeded modes against the oracle's per-pixel sum
(HEALPix layouts, ring lengths with large odd prime factors, lengths 2 mod 4, the shortest
ring, the largest rings, modes that alias), and the whole path (chains, plain and scanned,
then the synthesis) on HEALPix rings against the oracle's chains and sums, FP64 1e-10 and
FP32 1e-4 relative RMS per field and per ring (FP64 on the plan's own order-2 setup: 20 times the
oracle's own FP64 sensitivity on these grids, measured in the test, when above 1e-10); the pixels'
covariance against the addition theorem (statistical); graph-capture replays; argument checks."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_rms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4}


def _ring_plan(n_ring, phi0, ell_max, precision, order=1, kap=100.0, z=None):
    from paper_1709_10314_amd import RingPlan

    return RingPlan(order, n_ring, phi0, ell_max, kappa=[kap] * order, precision=precision, z=z)


def _modes(plan, count, seed):
    """Seeded modes in the plan's sample_modes layout (entries above m_top zero), and the
    same values as the oracle's complex array (rounded to the plan's type first)."""
    rng = np.random.default_rng(seed)
    mt = plan.m_top
    g = np.zeros((count, plan.n_theta, plan.n_phi // 2, 2))
    g[:, :, : mt + 1] = rng.standard_normal((count, plan.n_theta, mt + 1, 2))
    g[:, :, 0, 1] = 0.0
    dev = torch.tensor(g, dtype=plan.dtype(), device="cuda")
    gh = dev.double().cpu().numpy()[:, :, : mt + 1]
    return dev, gh[..., 0] + 1j * gh[..., 1]


def _check(tag, T, To, offsets, bar):
    worst = 0.0
    for f in range(T.shape[0]):
        e = rel_rms(T[f], To[f])
        er = max(rel_rms(T[f, offsets[i] : offsets[i + 1]], To[f, offsets[i] : offsets[i + 1]])
                 for i in range(len(offsets) - 1))
        worst = max(worst, e, er)
        log(f"{tag}: field {f} rel RMS {e:.3e}, worst ring {er:.3e}")
    assert worst <= bar


def _healpix(nside):
    from paper_1709_10314_amd import workloads

    return workloads.healpix_rings(nside)


# (name, ring lengths, phi0, ell_max)
def _layouts():
    rng = np.random.default_rng(7)
    out = []
    for nside in (1, 4, 16, 64):
        z, n_ring, phi0 = _healpix(nside)
        out.append((f"healpix-{nside}", n_ring, phi0, 3 * nside - 1))
    primes = np.array([2 * p for p in (3, 5, 7, 11, 13, 31, 127, 251, 509, 1021)], dtype=np.int32)
    out.append(("odd-primes", primes, rng.uniform(0, 2 * np.pi, len(primes)), 700))
    two_mod_4 = np.array([2, 6, 10, 18, 30, 42, 98, 2 * 243, 2 * 625, 2], dtype=np.int32)
    out.append(("two-mod-four", two_mod_4, rng.uniform(-1, 1, len(two_mod_4)), 1500))
    mixed = rng.integers(1, 1500, 24).astype(np.int32) * 2
    out.append(("random-even", mixed, rng.uniform(0, 7, len(mixed)), 400))
    return out


LAYOUTS = _layouts()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("layout", LAYOUTS, ids=lambda c: c[0])
def test_ring_synthesis_matches_oracle(layout, precision):
    name, n_ring, phi0, lmax = layout
    plan = _ring_plan(n_ring, phi0, lmax, precision)
    assert plan.m_top == lmax and plan.pixels == int(np.sum(n_ring))
    count = 2
    gdev, g = _modes(plan, count, seed=len(n_ring) + lmax)
    T = plan.synthesize_rings(gdev, count)
    torch.cuda.synchronize()
    T = T.double().cpu().numpy()
    To = oracle.dft_rings(g, n_ring, phi0)
    _check(f"{name} {precision}", T, To, plan.offsets, TOL[precision])
    plan.close()


@pytest.mark.parametrize("precision,n_max", [("fp32", 8192), ("fp64", 4096)])
def test_largest_rings_and_all_modes(precision, n_max):
    """The largest ring each precision takes, next to its neighbours in length and the
    shortest ring, with ell_max = 8191 (the most modes a ring plan holds: 16384 / 2 - 1)."""
    n_ring = np.array([n_max, n_max - 2, 2, n_max - 6, 4], dtype=np.int32)
    phi0 = np.array([0.0, 0.1, 0.2, np.pi / n_max, 1.0])
    plan = _ring_plan(n_ring, phi0, 8191, precision, kap=4.0)
    assert plan.n_phi == 16384 and plan.m_top == 8191
    gdev, g = _modes(plan, 1, seed=11)
    T = plan.synthesize_rings(gdev, 1)
    torch.cuda.synchronize()
    To = oracle.dft_rings(g, n_ring, phi0)
    _check(f"largest rings {precision}", T.double().cpu().numpy(), To, plan.offsets, TOL[precision])
    plan.close()


# Ring lengths of the power-of-two and Bluestein transform classes: n / 2 a power of two from
# 512 to 4096, and n / 2 with a large odd prime (even and odd half-lengths, Bluestein lengths
# 512 to 4096), next to lengths the general kernel keeps; ell_max = 3071 makes the modes
# alias on the rings shorter than 3072 pixels.
CLASS_RINGS = [1024, 2048, 4096, 8192, 2 * 257, 2 * 683, 2 * 1018, 2 * 1021, 2 * 1535, 2 * 2047, 2 * 1536, 2 * 750]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_power_of_two_and_bluestein_ring_classes(precision):
    n_max = 8192 if precision == "fp32" else 4096
    n_ring = np.array([n for n in CLASS_RINGS if n <= n_max], dtype=np.int32)
    phi0 = np.random.default_rng(3).uniform(0, 2 * np.pi, len(n_ring))
    phi0[0] = 0.0
    phi0[1] = np.pi / n_ring[1]
    plan = _ring_plan(n_ring, phi0, 3071, precision)
    count = 2
    gdev, g = _modes(plan, count, seed=29)
    T = plan.synthesize_rings(gdev, count)
    torch.cuda.synchronize()
    To = oracle.dft_rings(g, n_ring, phi0)
    _check(f"ring classes {precision}", T.double().cpu().numpy(), To, plan.offsets, TOL[precision])
    # the lognormal map as these kernels store the pixels: exp(0.1 + 0.5 T) of the same seed's field
    Tg = plan.sample_rings(4, count).double().cpu().numpy()
    Tl = plan.sample_rings_lognormal(4, count, 0.1, 0.5).double().cpu().numpy()
    torch.cuda.synchronize()
    el = rel_rms(Tl, np.exp(0.1 + 0.5 * Tg))
    log(f"ring classes {precision}: lognormal map rel RMS {el:.3e}")
    assert el <= (1e-13 if precision == "fp64" else 1e-6)
    plan.close()


# (nside, order, kappa_i, ell_max, factors).  Order 1 at ell_max = 3 nside - 1 (modes alias
# on every ring, the belt's n / 2 being 2 nside); order 2 on the plan's own factors keeps
# m_top near n_theta / 2 (higher modes are evanescent at the polar rings, where pivots sit
# next to the factorisation threshold), and on the oracle's factors also at 3 nside - 1.
E2E = [(4, 1, 100.0, 11, "own"), (16, 1, 400.0, 47, "own"), (8, 2, 900.0, 15, "own"),
       (32, 2, 2500.0, 63, "own"), (8, 2, 900.0, 23, "oracle"), (32, 2, 2500.0, 63, "oracle")]


def _grid_sensitivity(order, C, z, nphi, n_ring, phi0, seed, count):
    """The oracle's own FP64 sensitivity on a symmetric grid: the largest field change (rel
    RMS) that moving the northern z values by a random relative 2.2e-16 causes (three draws).
    Order 2 on HEALPix's uneven polar rings reaches ~1e-9, order 1 ~1e-14."""
    n = len(z)
    A, B = oracle.setup(order, C, n, nphi, z=z)
    T = oracle.dft_rings(oracle.sample_modes(order, n, A, B, seed, count), n_ring, phi0)
    h = (n + 1) // 2
    sens = 0.0
    for d in range(3):
        zn = z[:h] * (1 + 2.2e-16 * np.random.default_rng(d).standard_normal(h))
        zp = np.concatenate([zn, -zn[: n - h][::-1]])
        Ap, Bp = oracle.setup(order, C, n, nphi, z=zp)
        Tp = oracle.dft_rings(oracle.sample_modes(order, n, Ap, Bp, seed, count), n_ring, phi0)
        sens = max(sens, max(rel_rms(Tp[f], T[f]) for f in range(count)))
    return sens


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", E2E, ids=lambda c: "nside%d-M%d-k%g-l%d-%s" % c)
def test_healpix_fields_match_oracle(case, precision):
    nside, order, kap, lmax, factors = case
    z, n_ring, phi0 = _healpix(nside)
    n = len(z)
    count, seed = 2, 41
    plan = _ring_plan(n_ring, phi0, lmax, precision, order=order, kap=kap, z=z)
    assert plan.symmetric and plan.m_top == lmax
    C = oracle.spectrum([kap] * order, lmax)
    A, B = oracle.setup(order, C, n, plan.n_phi, z=z)
    bar = TOL[precision]
    if factors == "oracle":
        plan.set_factors(A, B)
    elif precision == "fp64":
        # the plan's own FP64 setup differs from the oracle's by rounding; the bar is the
        # larger of 1e-10 and 20 times what FP64-sized grid changes do to the oracle's fields
        sens = _grid_sensitivity(order, C, z, plan.n_phi, n_ring, phi0, seed, count)
        bar = max(bar, 20 * sens)
        log(f"{case}: oracle's FP64 sensitivity {sens:.3e}, bar {bar:.3e}")
    g = oracle.sample_modes(order, n, A, B, seed, count)
    To = oracle.dft_rings(g, n_ring, phi0)
    for blocks in (1, 4):
        plan.set_ring_blocks(blocks)
        T = plan.sample_rings(seed, count)
        torch.cuda.synchronize()
        _check(f"{case} {precision} blocks {plan.ring_blocks(count)}", T.double().cpu().numpy(), To,
               plan.offsets, bar)
    plan.close()


@pytest.mark.parametrize("order", [3, 4])
def test_healpix_higher_orders_on_oracle_factors(order):
    """Orders 3 and 4 on HEALPix rings: the ring plan's chains on the oracle's factors
    (smf_set_factors; the order-3/4 setup's FP64 sensitivity is covered by the regular-grid
    tests), then the synthesis, against the oracle: FP64 1e-10, FP32 1e-4."""
    z, n_ring, phi0 = _healpix(16)
    n, lmax, kap, count, seed = len(z), 47, 900.0, 2, 43
    C = oracle.spectrum([kap] * order, lmax)
    for precision in ("fp64", "fp32"):
        plan = _ring_plan(n_ring, phi0, lmax, precision, order=order, kap=kap, z=z)
        A, B = oracle.setup(order, C, n, plan.n_phi, z=z)
        plan.set_factors(A, B)
        To = oracle.dft_rings(oracle.sample_modes(order, n, A, B, seed, count), n_ring, phi0)
        for blocks in (1, 4):
            plan.set_ring_blocks(blocks)
            T = plan.sample_rings(seed, count)
            torch.cuda.synchronize()
            _check(f"order {order} {precision} blocks {plan.ring_blocks(count)}", T.double().cpu().numpy(), To,
                   plan.offsets, TOL[precision])
        plan.close()


def test_healpix_u_basis():
    """The U basis of Sec. 3 (order 2) on HEALPix rings: FP32 on the plan's own setup against
    the oracle's U-basis setup and samples (1e-4), FP64 on the oracle's factors (1e-10; the
    plan's own FP64 setup is logged, its sensitivity being that of the z basis)."""
    from paper_1709_10314_amd import RingPlan

    z, n_ring, phi0 = _healpix(8)
    n, lmax, kap, count, seed = len(z), 15, 900.0, 2, 47
    C = oracle.spectrum([kap, kap], lmax)
    for precision in ("fp64", "fp32"):
        plan = RingPlan(2, n_ring, phi0, lmax, kappa=[kap, kap], precision=precision, z=z, basis="u")
        A, B = oracle.setup(2, C, n, plan.n_phi, z=z, basis="u")
        To = oracle.dft_rings(oracle.sample_modes(2, n, A, B, seed, count), n_ring, phi0)
        T = plan.sample_rings(seed, count)
        torch.cuda.synchronize()
        T = T.double().cpu().numpy()
        if precision == "fp32":
            _check("u basis fp32, own setup", T, To, plan.offsets, TOL[precision])
        else:
            log(f"u basis fp64, own setup: {max(rel_rms(T[f], To[f]) for f in range(count)):.3e}")
            plan.set_factors(A, B)
            T = plan.sample_rings(seed, count)
            torch.cuda.synchronize()
            _check("u basis fp64, oracle factors", T.double().cpu().numpy(), To, plan.offsets, TOL[precision])
        plan.close()


def test_sample_rings_is_sample_modes_then_synthesis():
    z, n_ring, phi0 = _healpix(16)
    plan = _ring_plan(n_ring, phi0, 40, "fp32", order=2, kap=400.0, z=z)
    a = plan.sample_rings(5, 3).clone()
    g = plan.sample_modes(5, 3)
    b = plan.synthesize_rings(g, 3)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.close()


def test_ring_plan_arguments():
    from paper_1709_10314_amd import SmfError, smf

    z, n_ring, phi0 = _healpix(4)
    bad = {
        "odd ring": np.where(np.arange(len(n_ring)) == 3, 7, n_ring),
        "empty ring": np.where(np.arange(len(n_ring)) == 0, 0, n_ring),
        "ring too long": np.where(np.arange(len(n_ring)) == 5, 8194, n_ring),
    }
    for what, nr in bad.items():
        rc, _ = smf.smf_setup_rings(1, nr, phi0, 11, kappa=[30.0], flags=smf.SMF_FP32)
        assert rc == smf.SMF_EINVAL, what
    rc, _ = smf.smf_setup_rings(1, np.full(len(n_ring), 4096 + 2), phi0, 11, kappa=[30.0], flags=smf.SMF_FP64)
    assert rc == smf.SMF_EINVAL
    rc, _ = smf.smf_setup_rings(1, n_ring, np.where(np.arange(len(n_ring)) == 2, np.nan, phi0), 11,
                                kappa=[30.0], flags=smf.SMF_FP32)
    assert rc == smf.SMF_EINVAL
    rc, _ = smf.smf_setup_rings(1, n_ring, phi0, 8192, kappa=[30.0], flags=smf.SMF_FP32)
    assert rc == smf.SMF_EINVAL
    rc, _ = smf.smf_setup_rings(1, n_ring, phi0, 11, kappa=[30.0], flags=smf.SMF_FP32, z=z[::-1].copy())
    assert rc == smf.SMF_EINVAL
    plan = _ring_plan(n_ring, phi0, 11, "fp32", kap=30.0)
    assert plan.n_phi == 32 and np.array_equal(plan.offsets, oracle.ring_offsets(n_ring))
    work = plan.empty(2)
    assert smf.smf_sample_rings(plan.handle, 1, 2, work.data_ptr(), work.data_ptr()) == smf.SMF_EINVAL
    assert smf.smf_sample_rings(plan.handle, 1, -1, work.data_ptr(), 0) == smf.SMF_EINVAL
    assert smf.smf_sample_rings(plan.handle, 1, 0, 0, 0) == smf.SMF_OK
    rings = plan.empty_rings(1)
    assert smf.smf_synthesize_rings(plan.handle, 65536, work.data_ptr(), rings.data_ptr()) == smf.SMF_EINVAL
    with pytest.raises(ValueError):
        plan.sample_rings(1, 2, out=torch.empty(plan.pixels, device="cuda"))
    plan.close()
    from paper_1709_10314_amd import Plan

    p = Plan(1, 8, 16, 7, kappa=[30.0], precision="fp32")
    rc, _ = smf.smf_ring_layout(p.handle, 8)
    assert rc == smf.SMF_EINVAL
    assert smf.smf_synthesize_rings(p.handle, 1, p.empty(1).data_ptr(), p.empty(1).data_ptr()) == smf.SMF_EINVAL
    p.close()
    with pytest.raises(SmfError):
        _ring_plan(np.array([4]), np.array([0.0]), 3, "fp32")   # one ring: n_theta < 2


def test_sample_rings_graph_capture_replays():
    """smf_sample_rings (chains, then the ring launches, forked over the plan's streams and joined
    back) captured in a HIP graph: every replay, with eager work and synchronisations between
    replays, equals the eager call."""
    z, n_ring, phi0 = _healpix(32)
    n_ring = n_ring.copy()
    n_ring[3] = 2 * 509          # a Bluestein ring (L = 1024)
    n_ring[5] = 2048             # a power-of-two ring: three launches, two of them on the plan's streams
    plan = _ring_plan(n_ring, phi0, 95, "fp32", order=2, kap=900.0, z=z)
    eager = plan.sample_rings(13, 2).clone()
    torch.cuda.synchronize()
    out = plan.empty_rings(2)
    work = plan.empty(2)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.sample_rings(13, 2, out, work, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.sample_rings(13, 2, out, work, stream=s)
    for rep in range(3):
        out.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), rep
        del junk
    plan.close()


@pytest.mark.parametrize("order,kap", [(1, 10.0), (2, 30.0)])
def test_healpix_covariance_matches_addition_theorem(order, kap):
    """The law of the sampled pixels (Lemma 2.1 and the field covariance of Sec. 5): a ring plan
    keeps every mode, so the covariance of two pixels on one ring or on adjacent rings, which
    the chain reproduces exactly, is sum_l (2l+1)/(4 pi) C_l P_l(cos gamma).  200,000 FP64 fields
    on HEALPix nside 4: every such pixel pair within 5 standard errors (Isserlis), the means
    within 5 standard errors of 0."""
    from numpy.polynomial import legendre as npleg

    nside, lmax, n_fields, per_call = 4, 11, 200_000, 50_000
    z, n_ring, phi0 = _healpix(nside)
    plan = _ring_plan(n_ring, phi0, lmax, "fp64", order=order, kap=kap, z=z)
    out = plan.empty_rings(per_call)
    work = plan.empty(per_call)
    S = torch.zeros((plan.pixels, plan.pixels), dtype=torch.float64, device="cuda")
    mean = torch.zeros(plan.pixels, dtype=torch.float64, device="cuda")
    for c in range(n_fields // per_call):
        T = plan.sample_rings(1 + c * per_call, per_call, out, work)
        S += T.T @ T
        mean += T.sum(0)
    torch.cuda.synchronize()
    plan.close()
    S = (S / n_fields).cpu().numpy()
    mean = (mean / n_fields).cpu().numpy()
    C = oracle.spectrum([kap] * order, lmax)
    coef = (2 * np.arange(lmax + 1) + 1) / (4 * np.pi) * C
    ring = np.repeat(np.arange(len(z)), n_ring)
    phi = np.concatenate([phi0[i] + 2 * np.pi * np.arange(n_ring[i]) / n_ring[i] for i in range(len(z))])
    zp = z[ring]
    sp = np.sqrt((1 - zp) * (1 + zp))
    var = float(npleg.legval(1.0, coef))
    assert np.all(np.abs(mean) <= 5 * np.sqrt(var / n_fields))
    worst = 0.0
    pairs = 0
    for a in range(plan.pixels):
        b = np.nonzero(np.abs(ring - ring[a]) <= 1)[0]
        b = b[b >= a]
        cosg = np.clip(zp[a] * zp[b] + sp[a] * sp[b] * np.cos(phi[a] - phi[b]), -1.0, 1.0)
        target = npleg.legval(cosg, coef)
        se = np.sqrt((S[a, a] * S[b, b] + S[a, b] ** 2) / n_fields)
        worst = max(worst, float(np.max(np.abs(S[a, b] - target) / se)))
        pairs += len(b)
    log(f"order {order}: {pairs} pixel pairs, worst deviation {worst:.2f} standard errors; variance {var:.4e}")
    assert worst <= 5.0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ring_lognormal_is_exp_of_the_pixels(precision):
    """smf_sample_rings_lognormal stores exp(mu + sigma T) of the pixels smf_sample_rings gives
    (both launches: one ring takes the chirp-z pass), and against the oracle's pixels."""
    z, n_ring, phi0 = _healpix(16)
    n_ring = n_ring.copy()
    n_ring[5] = 2 * 509
    mu, sig, count, seed = 0.4, 3.0, 2, 17
    plan = _ring_plan(n_ring, phi0, 47, precision, order=1, kap=400.0, z=z)
    T = plan.sample_rings(seed, count).clone()
    L = plan.sample_rings_lognormal(seed, count, mu, sig)
    torch.cuda.synchronize()
    T = T.double().cpu().numpy()
    L = L.double().cpu().numpy()
    if precision == "fp64":
        ref = np.exp(mu + sig * T)
        bound = 1e-14
    else:
        y = np.float32(mu) + np.float32(sig) * T
        ref = np.exp(y)
        bound = 4 * 2.0 ** -24 + float(np.max(np.abs(y))) * 2.0 ** -24 * 2
    e = float(np.max(np.abs(L - ref) / ref))
    log(f"ring lognormal {precision}: max rel err vs exp(pixels) {e:.2e} (bound {bound:.2e})")
    assert e <= bound
    C = oracle.spectrum([400.0], 47)
    A, B = oracle.setup(1, C, len(z), plan.n_phi, z=z)
    To = oracle.dft_rings(oracle.sample_modes(1, len(z), A, B, seed, count), n_ring, phi0)
    for f in range(count):
        el = rel_rms(L[f], np.exp(mu + sig * To[f]))
        lim = TOL[precision] * max(1.0, sig * float(np.max(np.abs(To[f]))))
        log(f"  field {f}: lognormal rel RMS vs oracle {el:.2e} (limit {lim:.2e})")
        assert el <= lim
    from paper_1709_10314_amd import smf

    out, work = plan.empty_rings(1), plan.empty(1)
    for bad in (float("nan"), float("inf")):
        assert smf.smf_sample_rings_lognormal(plan.handle, 1, 1, bad, 1.0, work.data_ptr(),
                                              out.data_ptr()) == smf.SMF_EINVAL
        assert smf.smf_sample_rings_lognormal(plan.handle, 1, 1, 0.0, bad, work.data_ptr(),
                                              out.data_ptr()) == smf.SMF_EINVAL
    plan.close()


@pytest.mark.parametrize("precision,nside", [("fp32", 2048), ("fp64", 1024)])
def test_largest_healpix_plans_sampled_rings(precision, nside):
    """The largest HEALPix grid of each precision (FP32 nside 2048: 8191 rings, 8192-pixel belt
    rings, ell_max 6143, 50M pixels; FP64 nside 1024), order 2: the plan's own modes, synthesised
    on the GPU, against the oracle's per-pixel sum of the same modes on sampled rings (the
    poles, polar rings whose odd part is a large prime, both kinds of belt ring)."""
    z, n_ring, phi0 = _healpix(nside)
    lmax = 3 * nside - 1
    plan = _ring_plan(n_ring, phi0, lmax, precision, order=2, kap=2500.0, z=z)
    assert plan.pixels == 12 * nside * nside
    g = plan.sample_modes(5, 1)
    T = plan.synthesize_rings(g, 1)
    torch.cuda.synchronize()
    n = len(z)
    # polar ring i holds 4 (i + 1) pixels: half-lengths 2 (i + 1) that are powers of two (i = 255,
    # 511, 1023), that have a large odd prime (256: 257, 508: 509, 682: 683, 1020: 1021), or
    # small ones only (767: 3 x 256)
    picks = [0, 1, 2, nside // 2 - 1, 255, 256, 508, 511, 682, 767, 1020, 1023, nside - 2, nside - 1, nside,
             2 * nside - 1, 2 * nside, 3 * nside, n - 1021, n - 257, n - 2, n - 1]
    picks = sorted({i for i in picks if 0 <= i < n})
    gs = g[0, picks].double().cpu().numpy()[:, : lmax + 1]
    gs = (gs[..., 0] + 1j * gs[..., 1])[None]
    To = oracle.dft_rings(gs, n_ring[picks], phi0[picks])[0]
    off_o = oracle.ring_offsets(n_ring[picks])
    T = T[0].double().cpu().numpy()
    worst = 0.0
    for a, i in enumerate(picks):
        e = rel_rms(T[plan.offsets[i] : plan.offsets[i + 1]], To[off_o[a] : off_o[a + 1]])
        worst = max(worst, e)
    log(f"healpix nside {nside} {precision}: {len(picks)} sampled rings, worst rel RMS {worst:.3e}")
    assert worst <= TOL[precision]
    plan.close()
    del g, T
    torch.cuda.empty_cache()
