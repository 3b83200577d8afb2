"""Seeded synthetic workloads of the benchmark and the tests.

Only shapes, spectra parameters and seeds live here (no arithmetic of the method), so
both the HIP path and the oracle can be driven from the same definitions.  Spectra are
C_l = (l(l+1) + kappa^2)^-M, i.e. M repeated factors kappa_i = kappa^2 of eq. (Cl);
ell_max is the band limit of the Legendre sums.
"""
import math

import numpy as np

PLAIN_SMALL = dict(name="plain-64x128-M1-fp64", n_theta=64, n_phi=128, order=1, kappa=8.0,
                   ell_max=63, count=1, seed=1, precision="fp64")
PLAIN_1024 = dict(name="plain-1024x2048-M1-fp64-x16", n_theta=1024, n_phi=2048, order=1,
                  kappa=20.0, ell_max=1023, count=16, seed=1, precision="fp64")
PRECISION_4096 = dict(name="precision-4096x8192-M2-fp32-x8", n_theta=4096, n_phi=8192, order=2,
                      kappa=50.0, ell_max=4095, count=8, seed=1, precision="fp32")
PRECISION_8192 = dict(name="precision-8192x16384-M2-fp32-x4", n_theta=8192, n_phi=16384,
                      order=2, kappa=100.0, ell_max=8191, count=4, seed=1, precision="fp32")

CONFIGS = [PLAIN_SMALL, PLAIN_1024, PRECISION_4096, PRECISION_8192]


def kappas(cfg):
    """kappa_i of eq. (Cl) for a config: kappa^2 repeated `order` times."""
    return [cfg["kappa"] ** 2] * cfg["order"]


def batch_mix(n_fields=256, seed=0):
    """Mixed batch: n_theta uniform on {128, ..., 2048}, n_phi = 2 n_theta, ln kappa
    uniform on [ln 2, ln 200], order 1 or 2 with equal probability, ell_max = n_theta - 1,
    Philox seeds 1..n_fields.  Drawn with numpy's PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.array([128, 256, 512, 1024, 2048])
    out = []
    for f in range(n_fields):
        n_theta = int(rng.choice(sizes))
        kappa = float(math.exp(rng.uniform(math.log(2.0), math.log(200.0))))
        order = int(1 + rng.integers(0, 2))
        out.append(dict(n_theta=n_theta, n_phi=2 * n_theta, order=order, kappa=kappa,
                        ell_max=n_theta - 1, seed=1 + f, precision="fp32"))
    return out


# ---- ring grids z_0 > z_1 > ... > z_{n-1}, symmetric about the equator (z_{n-1-i} = -z_i
# exactly), the grid argument of Alg. 1 ----

def _mirror(z_north, n):
    """Full grid from its northern values z_0 .. z_{ceil(n/2)-1} (the middle one 0 for odd n)."""
    z = np.empty(n)
    h = (n + 1) // 2
    z[:h] = z_north[:h]
    if n % 2:
        z[h - 1] = 0.0
    z[n - h:] = -z[:h][::-1]
    return z


def gauss_legendre_z(n):
    """The n Gauss-Legendre nodes in (-1, 1), descending (numpy's leggauss)."""
    x = np.polynomial.legendre.leggauss(n)[0][::-1].copy()
    return _mirror(x, n)


def healpix_ring_z(nside):
    """The 4 nside - 1 ring latitudes of a HEALPix grid: z = 1 - k^2 / (3 nside^2) in the
    polar caps (k < nside), z = (4 nside - 2k) / (3 nside) in the equatorial belt."""
    k = np.arange(1, 2 * nside + 1, dtype=np.float64)
    zn = np.where(k < nside, 1.0 - k * k / (3.0 * nside * nside), (4.0 * nside - 2.0 * k) / (3.0 * nside))
    return _mirror(zn, 4 * nside - 1)


def random_z(n, seed=0):
    """A symmetric grid with the northern values drawn uniformly in (0, 1) (PCG64(seed))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = (n + 1) // 2
    zn = np.sort(rng.uniform(0.0, 1.0, h))[::-1]
    if n % 2 == 0:
        zn = np.maximum(zn, 1e-3)
    return _mirror(zn, n)


def random_asym_z(n, seed=0):
    """A grid with no symmetry: ring centres jittered independently by up to a fifth of a
    ring, z_i = cos(pi (i + 1/2 + u_i) / n), u_i uniform in (-0.2, 0.2) (PCG64(seed)), so
    neighbouring rings stay at least 0.6 of a spacing apart."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(-0.2, 0.2, n)
    return np.cos(np.pi * (np.arange(n) + 0.5 + u) / n)


def shifted_z(n, shift=0.3):
    """Ring centres shifted by a fraction of a ring: z_i = cos(pi (i + shift) / n), shift in (0, 1)."""
    return np.cos(np.pi * (np.arange(n) + shift) / n)


def healpix_rings(nside):
    """A HEALPix ring layout (Gorski et al. 2005, ApJ 622, 759): the 4 nside - 1 ring
    latitudes of healpix_ring_z, each ring k (1-based from the north) with its own pixel
    count and the longitude of its first pixel.  Polar rings (k < nside, and their mirrors)
    hold 4k pixels at phi_j = pi (j + 1/2) / (2k); belt rings hold 4 nside pixels at
    phi_j = pi (j + s/2) / (2 nside), s = (k - nside + 1) mod 2.  Returns (z, n_phi, phi0)
    with 12 nside^2 pixels in all."""
    n = 4 * nside - 1
    k = np.arange(1, n + 1)
    kk = np.minimum(k, 4 * nside - k)
    n_phi = np.where(kk < nside, 4 * kk, 4 * nside).astype(np.int32)
    s = (k - nside + 1) % 2
    phi0 = np.where(kk < nside, np.pi / (4.0 * kk), np.pi * s / (4.0 * nside))
    return healpix_ring_z(nside), n_phi, phi0.astype(np.float64)
