"""Pins of the oracle's synthesis on rings with their own pixel counts and first-pixel
longitudes (Alg. 2's last step on an iso-latitude grid such as HEALPix, Sec. 1), against
what fixes it independently of the oracle: numpy's inverse real FFT on equal rings with no
offset; a long inverse real FFT sampled at the ring's pixels for offsets that are rational
fractions of a pixel and for modes above n/2 (which alias); the closed form of a single
mode; and the HEALPix layout's published pixel counts and pixel centres."""
import numpy as np
import pytest

import oracle


def _modes(rng, count, n_theta, mt):
    g = rng.standard_normal((count, n_theta, mt + 1)) + 1j * rng.standard_normal((count, n_theta, mt + 1))
    g[..., 0] = g[..., 0].real
    return g


def test_equal_rings_without_offset_are_numpy_irfft():
    rng = np.random.default_rng(1)
    n, mt = 32, 15
    g = _modes(rng, 2, 5, mt)
    T = oracle.dft_rings(g, [n] * 5, np.zeros(5)).reshape(2, 5, n)
    full = np.zeros((2, 5, n // 2 + 1), complex)
    full[..., : mt + 1] = g
    ref = np.fft.irfft(full, n=n, axis=-1) * n
    assert np.abs(T - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("n,mt,p,q", [(12, 5, 1, 2), (12, 17, 1, 2), (20, 45, 1, 4), (4, 9, 0, 1),
                                      (36, 40, 3, 8), (8, 3, 1, 2), (60, 7, 2, 3)])
def test_offsets_and_aliasing_against_sampled_long_irfft(n, mt, p, q):
    """phi_j = 2 pi (j + p/q) / n is pixel (p + q j) K of an inverse real FFT of length
    L = q n K, which holds every mode when L > 2 m_top."""
    rng = np.random.default_rng(n * 100 + mt)
    g = _modes(rng, 1, 1, mt)
    T = oracle.dft_rings(g, [n], [2 * np.pi * p / (q * n)])[0]
    K = 1
    while q * n * K <= 2 * mt + 1:
        K += 1
    L = q * n * K
    full = np.zeros(L // 2 + 1, complex)
    full[: mt + 1] = g[0, 0]
    ref = (np.fft.irfft(full, n=L) * L)[(p + q * np.arange(n)) * K]
    assert np.abs(T - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("m", [0, 1, 3, 5, 7, 11, 25])
def test_single_mode_closed_form(m):
    """g_m = a + i b, all other modes 0: T_j = 2 (a cos(m phi_j) - b sin(m phi_j)) for m > 0,
    a for m = 0; ring of 10 pixels offset by 0.3 rad (m = 7, 11, 25 alias)."""
    n, phi0, a, b = 10, 0.3, 0.7, -1.3
    g = np.zeros((1, 1, 26), complex)
    g[0, 0, m] = a if m == 0 else a + 1j * b
    T = oracle.dft_rings(g, [n], [phi0])[0]
    phi = phi0 + 2 * np.pi * np.arange(n) / n
    ref = np.full(n, a) if m == 0 else 2 * (a * np.cos(m * phi) - b * np.sin(m * phi))
    assert np.abs(T - ref).max() <= 1e-13


def test_rings_are_independent_and_laid_out_by_offsets():
    rng = np.random.default_rng(3)
    n_ring = np.array([4, 8, 12, 8, 4])
    phi0 = np.array([0.1, 0.0, 0.5, 1.0, 2.0])
    g = _modes(rng, 2, 5, 9)
    T = oracle.dft_rings(g, n_ring, phi0)
    off = oracle.ring_offsets(n_ring)
    assert T.shape == (2, off[-1]) and off[-1] == 36
    for f in range(2):
        for i in range(5):
            one = oracle.dft_rings(g[f : f + 1, i : i + 1], n_ring[i : i + 1], phi0[i : i + 1])[0]
            assert np.array_equal(T[f, off[i] : off[i + 1]], one)


@pytest.mark.parametrize("nside", [1, 2, 4, 16, 64])
def test_healpix_layout(nside):
    """12 nside^2 pixels on 4 nside - 1 rings; pixel centres of the belt lie on the
    longitudes pi (j + s/2) / (2 nside); every ring is equally spaced and symmetric in z."""
    from paper_1709_10314_amd import workloads

    z, n_ring, phi0 = workloads.healpix_rings(nside)
    assert len(z) == len(n_ring) == len(phi0) == 4 * nside - 1
    assert n_ring.sum() == 12 * nside * nside
    assert np.array_equal(n_ring, n_ring[::-1]) and np.allclose(z, -z[::-1], rtol=0, atol=1e-15)
    assert np.all(n_ring % 4 == 0) and n_ring.max() == 4 * nside
    # the caps: ring k has 4k pixels, the first at pi / (4k)
    k = np.arange(1, nside)
    assert np.array_equal(n_ring[: nside - 1], 4 * k)
    np.testing.assert_allclose(phi0[: nside - 1], np.pi / (4 * k), rtol=1e-15)
    # the belt alternates between a half-pixel offset (its first ring) and none
    belt = phi0[nside - 1 : 3 * nside]
    np.testing.assert_allclose(belt[0::2], np.pi / (4 * nside), rtol=1e-15)
    assert np.all(belt[1::2] == 0.0)
