"""The largest plan the C ABI accepts: n_theta = 65536 rings, n_phi = 16384, order 2, one
field (4.3 GB of FP32 output, 8.6 GB in FP64; 26 GB of factors), ell_max = 63 so that the
setup stays short.  This checks the 64-bit offsets of rings, fields and factor sets, the
plain recursion and the affine scan over a 32,767-step walk, and the FFT at its largest
size.

At ell_max = 63 these 65536 rings oversample the field about a thousandfold: every step's
transition is A = I + O(5e-5), whose departure from I FP32 holds to only ~1e-3, and whose
FP64 rounding differs between two setups enough for their chains to drift apart by ~1e-9
over the walk.  The chains are therefore compared on the oracle's own factors
(smf_set_factors), sampled modes over every ring and sampled rings against numpy's inverse
real FFT of the GPU's modes of those rings: FP64 (plain and scanned) against the oracle's
chains at 1e-10; the FP32 plain walk against the oracle's FP64 chains run on the same
factors rounded to FP32 (the values the FP32 plan steps with) at 1e-4; the FP32 scan, whose
block transitions are products of the FP64 factors, against the oracle's chains on the FP64
factors at 1e-4."""
import numpy as np
import pytest

import oracle
from gpu_helpers import log, rel_rms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4}
N, NPHI, LMAX, KAP = 65536, 16384, 63, 900.0
MODES = [0, 1, 17, 40, 63]
RINGS = [0, 1, 5000, 32766, 32767, 32768, 50000, 65534, 65535]
SEED = 2


def _oracle_factors():
    C = oracle.spectrum([KAP, KAP], LMAX)
    return oracle.setup(2, C, N, NPHI)


def _gpu_modes_and_rings(plan):
    g = plan.sample_modes(SEED, 1)
    torch.cuda.synchronize()
    gm = g[0][:, MODES, :].double().cpu().numpy()
    gr = g[0][RINGS][:, : LMAX + 1, :].double().cpu().numpy()
    del g
    T = plan.sample(SEED, 1)
    torch.cuda.synchronize()
    Tr = T[0][RINGS].double().cpu().numpy()
    del T
    return gm[..., 0] + 1j * gm[..., 1], gr[..., 0] + 1j * gr[..., 1], Tr


def _check(tag, gm, gr, Tr, go, bar):
    e = rel_rms(np.stack([gm.real, gm.imag]), np.stack([go.real, go.imag]))
    full = np.zeros((len(RINGS), NPHI // 2 + 1), dtype=np.complex128)
    full[:, : LMAX + 1] = gr
    full[:, 0] = full[:, 0].real
    ref = np.fft.irfft(full, n=NPHI, axis=1) * NPHI
    eT = max(rel_rms(Tr[i], ref[i]) for i in range(len(RINGS)))
    log(f"  {tag}: sampled modes over all rings {e:.3e}; sampled rings vs inverse FFT {eT:.3e}")
    assert e <= bar and eT <= bar


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_maximum_size_plan(precision):
    from paper_1709_10314_amd import Plan

    log(f"max size {N}x{NPHI} {precision}: oracle factors")
    A, B = _oracle_factors()
    go = oracle.sample_modes_list(2, N, MODES, A[:, MODES], B[:, MODES], SEED, 1)[0]
    refs = {0: go, 1: go}
    if precision == "fp32":
        A32, B32 = (X[:, MODES].astype(np.float32).astype(np.float64) for X in (A, B))
        refs[1] = oracle.sample_modes_list(2, N, MODES, A32, B32, SEED, 1)[0]
    log("  GPU setup")
    plan = Plan(2, N, NPHI, LMAX, kappa=[KAP, KAP], precision=precision)
    plan.set_factors(A, B)
    for blocks in (0, 1):
        plan.set_ring_blocks(blocks)
        assert (plan.ring_blocks(1) > 1) == (blocks == 0)
        gm, gr, Tr = _gpu_modes_and_rings(plan)
        _check(f"oracle factors, ring blocks {plan.ring_blocks(1)}", gm, gr, Tr, refs[blocks], TOL[precision])
    plan.close()
    torch.cuda.empty_cache()
