"""GPU parity on explicit ring grids (Alg. 1 takes the grid z as an input; symmetric grids
store the northern half, the remark after Alg. 1): Gauss-Legendre nodes, HEALPix ring
latitudes and random symmetric grids, even and odd ring counts, both orders; and grids with
no symmetry (random and shifted ring centres), whose southern walk has its own factor sets.  Factors
against the oracle's explicit-grid setup (by their action on the chain's law, as for the
ring-centre grid), modes and fields against the oracle on the same Philox normals (FP64
1e-10, FP32 1e-4 relative RMS per field, plain recursion and affine scan), the ring-centre
grid given as values against smf_setup, and the grid checks of smf_setup_grid."""
import numpy as np
import pytest

import oracle
from gpu_helpers import factor_errors, log, rel_rms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4}


def _grid(name):
    from paper_1709_10314_amd import workloads as w

    kind, n = name.rsplit("-", 1)
    n = int(n)
    if kind == "gl":
        return w.gauss_legendre_z(n)
    if kind == "healpix":
        return w.healpix_ring_z(n)
    return w.random_z(n, seed=n)


# (grid, order, kappa_i, n_phi, ell_max).  Order-2 cases keep m_top near n_theta / 2 or
# below: modes far above that are evanescent at the polar rings, where many pivots sit next
# to the factorisation threshold on either side (the ring-centre grid behaves the same).
CASES = [
    ("gl-64", 1, 400.0, 128, 63),
    ("gl-65", 2, 900.0, 64, 64),
    ("healpix-16", 1, 100.0, 128, 63),
    ("healpix-16", 2, 2500.0, 64, 70),
    ("healpix-32", 2, 900.0, 128, 127),
    ("random-100", 1, 50.0, 256, 99),
    ("random-37", 1, 9.0, 64, 20),
    ("gl-256", 2, 2500.0, 128, 255),
]


def _plan(z, order, kap, nphi, lmax, precision):
    from paper_1709_10314_amd import Plan

    return Plan(order, len(z), nphi, lmax, kappa=[kap] * order, precision=precision, z=z)


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-M%d-k%g-%d-l%d" % c)
def test_grid_factors_match_oracle(case):
    name, order, kap, nphi, lmax = case
    z = _grid(name)
    n = len(z)
    log(f"grid factors {case}")
    plan = _plan(z, order, kap, nphi, lmax, "fp64")
    Ag, Bg = plan.factors()
    plan.close()
    C = oracle.spectrum([kap] * order, lmax)
    Ao, Bo = oracle.setup(order, C, n, nphi, z=z)
    dA, dB, amb = factor_errors(Ag, Bg, Ao, Bo, n)
    log(f"  max dA {dA:.3e}  max dB {dB:.3e}  ({amb} steps next to a threshold)")
    assert dA < 1e-8 and dB < 1e-9
    assert amb <= max(2, 0.02 * Ao.shape[0] * Ao.shape[1])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-M%d-k%g-%d-l%d" % c)
def test_grid_modes_and_field_match_oracle(case, precision):
    name, order, kap, nphi, lmax = case
    z = _grid(name)
    n = len(z)
    count, seed = 2, 29
    C = oracle.spectrum([kap] * order, lmax)
    A, B = oracle.setup(order, C, n, nphi, z=z)
    To, go = oracle.sample(order, n, nphi, A, B, seed, count)
    plan = _plan(z, order, kap, nphi, lmax, precision)
    mt = plan.m_top
    for blocks in (1, 4):
        plan.set_ring_blocks(blocks)
        used = plan.ring_blocks(count)
        g = plan.sample_modes(seed, count)
        torch.cuda.synchronize()
        g = g.double().cpu().numpy()
        g = g[..., 0] + 1j * g[..., 1]
        T = plan.sample(seed, count)
        torch.cuda.synchronize()
        T = T.double().cpu().numpy()
        for f in range(count):
            eg = rel_rms(np.stack([g[f, :, : mt + 1].real, g[f, :, : mt + 1].imag]),
                         np.stack([go[f].real, go[f].imag]))
            eT = rel_rms(T[f], To[f])
            log(f"{case} {precision} blocks {used}: field {f} modes {eg:.3e} field {eT:.3e}")
            assert eg <= TOL[precision] and eT <= TOL[precision]
    plan.close()


@pytest.mark.parametrize("n", [64, 65])
def test_ring_centre_grid_as_values_matches_default(n):
    """The ring centres passed as values give the fields of smf_setup (the two setups differ
    only in how sin(theta) is rounded)."""
    from paper_1709_10314_amd import Plan

    z = oracle.grid(n)[1]
    a = Plan(2, n, 128, 63, kappa=[400.0, 400.0], precision="fp64")
    b = Plan(2, n, 128, 63, kappa=[400.0, 400.0], precision="fp64", z=z)
    Ta = a.sample(3, 2).clone()
    Tb = b.sample(3, 2)
    torch.cuda.synchronize()
    e = max(rel_rms(Tb[f].cpu().numpy(), Ta[f].cpu().numpy()) for f in range(2))
    log(f"ring centres as values, n {n}: rel RMS {e:.2e}")
    assert e <= 1e-10
    a.close()
    b.close()


def test_setup_grid_rejects_bad_grids():
    from paper_1709_10314_amd import smf

    z = oracle.grid(8)[1]
    bad = {
        "ascending": z[::-1].copy(),
        "touches the poles": np.linspace(1.0, -1.0, 8),
        "not monotone": np.r_[z[:4], -z[:4]],
        "nan": np.where(np.arange(8) == 2, np.nan, z),
    }
    for what, zb in bad.items():
        rc, _ = smf.smf_setup(1, 8, 16, 7, kappa=[30.0], flags=smf.SMF_FP64, z=zb)
        assert rc == smf.SMF_EINVAL, what
    rc, _ = smf.smf_setup(1, 8, 16, 7, kappa=[30.0], flags=smf.SMF_FP64, z=z[:7])
    assert rc == smf.SMF_EINVAL
    lib = smf.load()
    spec = smf.smf_spectrum()
    spec.order, spec.ell_max, spec.n_kappa = 1, 7, 0
    c = np.ones(8)
    spec.c_ell = c.ctypes.data_as(smf.ctypes.POINTER(smf.ctypes.c_double))
    h = smf.ctypes.c_void_p()
    assert lib.smf_setup_grid(smf.ctypes.byref(spec), 8, None, 16, smf.SMF_FP64, None,
                              smf.ctypes.byref(h)) == smf.SMF_EINVAL


# ---- grids with no symmetry: the south walks its own factor sets
ASYM = [
    ("asym-40", 2, 900.0, 64, 39),
    ("asym-41", 1, 100.0, 64, 30),
    ("shift-64", 2, 2500.0, 64, 63),
    ("shift-65", 1, 400.0, 128, 64),
    ("shift-130", 2, 700.0, 128, 129),
]


def _asym_grid(name):
    from paper_1709_10314_amd import workloads as w

    kind, n = name.rsplit("-", 1)
    n = int(n)
    return w.random_asym_z(n, seed=n) if kind == "asym" else w.shifted_z(n, 0.3)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ASYM, ids=lambda c: "%s-M%d-k%g-%d-l%d" % c)
def test_asymmetric_grid_matches_oracle(case, precision):
    """Modes and fields on a grid with no symmetry against the oracle's sampler with the
    southern walk's own sets (true coordinates), plain recursion and affine scan; the plan
    reports its grid and its asymmetry."""
    name, order, kap, nphi, lmax = case
    z = _asym_grid(name)
    n = len(z)
    count, seed = 2, 37
    C = oracle.spectrum([kap] * order, lmax)
    A, B, As, Bs = oracle.setup_asym(order, C, n, nphi, z)
    To, go = oracle.sample(order, n, nphi, A, B, seed, count, south=(As, Bs))
    plan = _plan(z, order, kap, nphi, lmax, precision)
    assert not plan.symmetric and np.array_equal(plan.z, z)
    mt = plan.m_top
    for blocks in (1, 4):
        plan.set_ring_blocks(blocks)
        used = plan.ring_blocks(count)
        g = plan.sample_modes(seed, count)
        torch.cuda.synchronize()
        g = g.double().cpu().numpy()
        g = g[..., 0] + 1j * g[..., 1]
        T = plan.sample(seed, count)
        torch.cuda.synchronize()
        T = T.double().cpu().numpy()
        for f in range(count):
            eg = rel_rms(np.stack([g[f, :, : mt + 1].real, g[f, :, : mt + 1].imag]),
                         np.stack([go[f].real, go[f].imag]))
            eT = rel_rms(T[f], To[f])
            log(f"{case} {precision} blocks {used}: field {f} modes {eg:.3e} field {eT:.3e}")
            assert eg <= TOL[precision] and eT <= TOL[precision]
    plan.close()


@pytest.mark.parametrize("case", ASYM[:3], ids=lambda c: "%s-M%d-k%g-%d-l%d" % c)
def test_asymmetric_grid_factors_round_trip_and_oracle_factors(case):
    """The plan's 2 n_sets factor sets (northern, then the southern walk's in true
    coordinates) against the oracle's entry by entry where they are well determined, and
    the sampler on the oracle's factors (smf_set_factors) against the oracle's samples."""
    name, order, kap, nphi, lmax = case
    z = _asym_grid(name)
    n = len(z)
    C = oracle.spectrum([kap] * order, lmax)
    A, B, As, Bs = oracle.setup_asym(order, C, n, nphi, z)
    plan = _plan(z, order, kap, nphi, lmax, "fp64")
    Ag, Bg = plan.factors()
    ns = plan.n_sets
    assert Ag.shape[0] == 2 * ns
    for Xg, Xo in ((Ag[:ns], A), (Bg[:ns], B), (Ag[ns:], As), (Bg[ns:], Bs)):
        big = np.abs(Xo) > 1e-6 * np.abs(Xo).max()
        e = float(np.max(np.abs(Xg - Xo)[big] / np.abs(Xo)[big]))
        log(f"{case}: factor entries rel err {e:.2e}")
        assert e < 1e-6
    plan.set_factors(np.concatenate([A, As]), np.concatenate([B, Bs]))
    T = plan.sample(3, 2)
    torch.cuda.synchronize()
    T = T.cpu().numpy()
    plan.close()
    To, _ = oracle.sample(order, n, nphi, A, B, 3, 2, south=(As, Bs))
    e = max(rel_rms(T[f], To[f]) for f in range(2))
    log(f"{case}: sampler on the oracle's factors {e:.3e}")
    assert e <= 1e-12


def test_symmetric_grid_reports_mirror():
    from paper_1709_10314_amd import Plan, workloads

    z = workloads.gauss_legendre_z(32)
    p = Plan(2, 32, 64, 31, kappa=[100.0, 100.0], precision="fp64", z=z)
    assert p.symmetric and np.array_equal(p.z, z) and p.factors()[0].shape[0] == p.n_sets
    p.close()
    q = Plan(2, 32, 64, 31, kappa=[100.0, 100.0], precision="fp64")
    assert q.symmetric
    np.testing.assert_allclose(q.z, oracle.grid(32)[1], rtol=0, atol=1e-15)
    q.close()


@pytest.mark.parametrize("order,n,precision", [(1, 64, "fp64"), (2, 64, "fp32"), (2, 33, "fp64"), (2, 128, "fp32")])
def test_no_mirror_plan_stores_southern_sets_and_samples_the_same(order, n, precision):
    """SMF_NO_MIRROR: the plan holds the southern walk's own sets (true coordinates); on the
    ring-centre grid, symmetric to the bit, they are the mirror D A D, D B D of the northern
    ones exactly, and the samples equal the mirrored plan's bit for bit, and the oracle's."""
    from paper_1709_10314_amd import Plan

    nphi, lmax = 1 << (2 * n - 1).bit_length(), n - 1
    kap = [40.0] * order
    pm = Plan(order, n, nphi, lmax, kappa=kap, precision=precision)
    pn = Plan(order, n, nphi, lmax, kappa=kap, precision=precision, mirror=False)
    assert pm.symmetric and not pn.symmetric
    Am, Bm = pm.factors()
    An, Bn = pn.factors()
    ns = pm.n_sets
    assert An.shape[0] == 2 * ns
    np.testing.assert_array_equal(An[:ns], Am)
    np.testing.assert_array_equal(Bn[:ns], Bm)
    j0 = 2 if n % 2 == 0 else 1
    D = np.diag([(-1.0) ** p for p in range(order)])
    np.testing.assert_array_equal(An[ns + j0:], D @ Am[j0:] @ D)
    np.testing.assert_array_equal(Bn[ns + j0:], D @ Bm[j0:] @ D)
    Tm = pm.sample(5, 3).double().cpu().numpy()
    Tn = pn.sample(5, 3).double().cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(Tm, Tn)
    C = oracle.spectrum(kap, lmax)
    A, B = oracle.setup(order, C, n, nphi)
    To, _ = oracle.sample(order, n, nphi, A, B, 5, 3)
    e = max(rel_rms(Tn[f], To[f]) for f in range(3))
    log(f"no-mirror {order} {n} {precision}: vs oracle {e:.2e}")
    assert e <= (1e-10 if precision == "fp64" else 1e-4)
    pm.close()
    pn.close()
