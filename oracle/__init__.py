"""FP64 CPU oracle for the sphere GRF sampler (Creasey & Lang, arXiv:1709.10314).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the product library never does.

The arithmetic lives in ``oracle.c`` (plain C, FP64, OpenMP); this module only builds
it with gcc and marshals numpy arrays through ctypes.  Functions and the passages of
the paper they follow:

* ``grid``          -- ring-centre grid (Sec. 4 grid, read as ring centres)
* ``spectrum``      -- C_l = prod_i (kappa_i + l(l+1))^-1           (eq. (Cl))
* ``spectrum_complex`` -- the same with complex kappa_i in conjugate pairs (Sec. 3)
* ``legendre``      -- L_lm(z) and dL_lm/dz                          (Sec. 2)
* ``jblock``        -- J^m_pq(z1, z2), brute-force sum over l        (Lemma 2.1)
* ``green_G``, ``green_P``, ``jblock_green``, ``setup_green``
                    -- order 1 without band limit: J^m from the Green's function,
                       P^m_lambda of complex degree by its hypergeometric series
                       (Sec. 3; eqs. (Legendre_hypergeometric), (Jmatrix_efficient))
* ``setup``         -- A, B, B_eq per mode and ring step             (Alg. 1; eqs.
                       (trans_matrix), (innov_matrix), (state_initial))
* ``philox``/``normal`` -- white-noise source (Philox4x32-10 + Box-Muller)
* ``sample_modes``  -- the state-space recursion, both hemispheres   (Alg. 2; eq. (state_space))
* ``dft``           -- inverse DFT along phi                         (Alg. 2, last step)
* ``dft_rings``     -- the same sum at the pixels of rings with their own pixel
                       counts and offsets (iso-latitude grids such as HEALPix, Sec. 1)
"""
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.c_double
_i = ctypes.c_int
_u64 = ctypes.c_uint64
_pd = ctypes.POINTER(ctypes.c_double)
_pu32 = ctypes.POINTER(ctypes.c_uint32)


def build(force=True):
    """Compile oracle.c into liboracle.so with gcc (IEEE FP64, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.orc_grid.argtypes = [_i, _pd, _pd]
    lib.orc_spectrum.argtypes = [_i, _pd, _i, _pd]
    lib.orc_spectrum.restype = _i
    lib.orc_spectrum_complex.argtypes = [_i, _pd, _pd, _i, _pd]
    lib.orc_spectrum_complex.restype = _i
    lib.orc_legendre.argtypes = [_i, _i, _d, _pd, _pd]
    lib.orc_jblock.argtypes = [_i, _i, _i, _pd, _d, _d, _pd]
    lib.orc_legendre_derivs.argtypes = [_i, _i, _d, _d, _i, ctypes.POINTER(_pd)]
    lib.orc_jblock_zs.argtypes = [_i, _i, _i, _pd, _d, _d, _d, _d, _pd]
    lib.orc_ring_zs.argtypes = [_i, _i, _pd, _pd]
    lib.orc_setup.argtypes = [_i, _i, _pd, _i, _i, _i, _pd, _pd]
    lib.orc_greenc_G.argtypes = [_i, _d, _d, _d, _d, _pd]
    lib.orc_greenc_G.restype = None
    lib.orc_jblock_green2c.argtypes = [_i, _pd, _d, _d, _d, _d, _pd]
    lib.orc_jblock_green2c.restype = None
    lib.orc_setup.restype = _i
    lib.orc_setup_z.argtypes = [_i, _i, _pd, _i, _pd, _i, _i, _pd, _pd]
    lib.orc_setup_z.restype = _i
    lib.orc_n_sets.argtypes = [_i]
    lib.orc_n_sets.restype = _i
    lib.orc_start_ring.argtypes = [_i]
    lib.orc_start_ring.restype = _i
    lib.orc_m_top.argtypes = [_i, _i]
    lib.orc_m_top.restype = _i
    lib.orc_philox.argtypes = [_pu32, _pu32, _pu32]
    lib.orc_normal.argtypes = [_u64, _i, _i, _i, _i, _i]
    lib.orc_normal.restype = _d
    lib.orc_sample_modes.argtypes = [_i, _i, _i, _i, _pd, _pd, _u64, _i, _pd]
    lib.orc_sample_modes.restype = _i
    _pi = ctypes.POINTER(ctypes.c_int)
    lib.orc_setup_modes.argtypes = [_i, _i, _pd, _i, _i, _pi, _i, _pd, _pd]
    lib.orc_setup_modes_z.argtypes = [_i, _i, _pd, _i, _pd, _i, _pi, _i, _pd, _pd]
    lib.orc_setup_modes_z.restype = _i
    lib.orc_setup_modes_asym.argtypes = [_i, _i, _pd, _i, _pd, _i, _pi, _i, _pd, _pd, _pd, _pd]
    lib.orc_setup_modes_zb.argtypes = [_i, _i, _i, _pd, _i, _pd, _i, _pi, _i, _pd, _pd]
    lib.orc_setup_modes_zb.restype = _i
    lib.orc_jblock_zs_u.argtypes = [_i, _i, _pd, _d, _d, _d, _d, _pd]
    lib.orc_setup_modes_asym.restype = _i
    lib.orc_setup_modes_asym_b.argtypes = [_i, _i, _i, _pd, _i, _pd, _i, _pi, _i, _pd, _pd, _pd, _pd]
    lib.orc_setup_modes_asym_b.restype = _i
    lib.orc_sample_modes_list_south.argtypes = [_i, _i, _pi, _i, _i, _pd, _pd, _pd, _pd, _u64, _i, _pd]
    lib.orc_sample_modes_list_south.restype = _i
    lib.orc_setup_modes.restype = _i
    lib.orc_sample_modes_list.argtypes = [_i, _i, _pi, _i, _i, _pd, _pd, _u64, _i, _pd]
    lib.orc_sample_modes_list.restype = _i
    lib.orc_dft.argtypes = [_i, _i, _i, _i, _i, _i, _pd, _pd]
    lib.orc_dft.restype = _i
    lib.orc_dft_rings.argtypes = [_i, _i, _i, _pi, _pd, ctypes.POINTER(ctypes.c_int64), _pd, _pd]
    lib.orc_dft_rings.restype = _i
    lib.orc_green_G.argtypes = [_i, _d, _d, _d]
    lib.orc_green_G.restype = _d
    lib.orc_green_P.argtypes = [_i, _d, _d, _d]
    lib.orc_green_P.restype = _d
    lib.orc_jblock_green.argtypes = [_i, _d, _d, _d, _d, _d, _pd]
    lib.orc_jblock_green2.argtypes = [_i, _pd, _d, _d, _d, _d, _pd]
    lib.orc_max_threads.restype = _i
    lib.orc_set_threads.argtypes = [_i]
    lib.orc_set_threads.restype = None
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(_pd)


def grid(n_theta):
    """theta_i = pi (i + 1/2) / n_theta and z_i = cos(theta_i), ring 0 nearest z = +1."""
    th = np.empty(n_theta)
    z = np.empty(n_theta)
    _load().orc_grid(n_theta, _p(th), _p(z))
    return th, z


def spectrum(kappa, ell_max):
    """C_l = prod_i (kappa_i + l(l+1))^-1, l = 0..ell_max (eq. (Cl))."""
    k = np.ascontiguousarray(kappa, dtype=np.float64).reshape(-1)
    C = np.empty(ell_max + 1)
    rc = _load().orc_spectrum(len(k), _p(k), ell_max, _p(C))
    if rc != 0:
        raise ValueError("spectrum has a non-positive or non-finite C_l")
    return C


def spectrum_complex(kappa, ell_max):
    """C_l = prod_i (kappa_i + l(l+1))^-1 with complex kappa_i (conjugate pairs, Sec. 3),
    l = 0..ell_max; the product must be real and positive."""
    k = np.asarray(kappa, dtype=np.complex128).reshape(-1)
    kre = np.ascontiguousarray(k.real)
    kim = np.ascontiguousarray(k.imag)
    C = np.empty(ell_max + 1)
    rc = _load().orc_spectrum_complex(len(k), _p(kre), _p(kim), ell_max, _p(C))
    if rc != 0:
        raise ValueError("spectrum has a C_l that is not real and positive")
    return C


def legendre(m, ell_max, theta):
    """(L, dL): L_lm(cos theta) and dL_lm/dz for l = m..ell_max (no Condon-Shortley sign)."""
    n = max(ell_max - m + 1, 0)
    L = np.zeros(n)
    dL = np.zeros(n)
    if n:
        _load().orc_legendre(m, ell_max, float(theta), _p(L), _p(dL))
    return L, dL


def legendre_derivs(m, ell_max, z, nd):
    """d^k L_lm / dz^k at z for k < nd (nd <= 4) and l = m..ell_max, as an [nd, n] array
    (k >= 2 from the associated Legendre equation)."""
    n = max(ell_max - m + 1, 0)
    F = np.zeros((4, max(n, 1)))
    if n:
        s = math.sqrt((1.0 - z) * (1.0 + z))
        ptrs = (ctypes.POINTER(ctypes.c_double) * 4)(*[F[k].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                                                        for k in range(4)])
        _load().orc_legendre_derivs(m, ell_max, float(z), s, nd, ptrs)
    return F[:nd, :n]


def jblock(order, m, ell_max, C, theta1, theta2):
    """J^m_pq(z1, z2) = sum_l C_l d^p L_lm(z1) d^q L_lm(z2), an order x order array."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    J = np.zeros(order * order)
    _load().orc_jblock(order, m, ell_max, _p(C), float(theta1), float(theta2), _p(J))
    return J.reshape(order, order)


def jblock_z(order, m, ell_max, C, z1, z2):
    """J^m(z1, z2) at two grid values, sin(theta) = sqrt((1 - z)(1 + z)) as the explicit-grid
    setup takes it."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    s1 = math.sqrt((1.0 - z1) * (1.0 + z1))
    s2 = math.sqrt((1.0 - z2) * (1.0 + z2))
    J = np.zeros(order * order)
    _load().orc_jblock_zs(order, m, ell_max, _p(C), float(z1), s1, float(z2), s2, _p(J))
    return J.reshape(order, order)


def _zs(z):
    return float(z), math.sqrt((1.0 - z) * (1.0 + z))


def green_G(m, kappa, z, s=None):
    """G_m(z) = 2F1(-lambda, lambda+1; 1+m; (1-z)/2) with kappa = -lambda(lambda+1) (Sec. 3)."""
    z, s0 = _zs(z)
    return _load().orc_green_G(int(m), float(kappa), z, s0 if s is None else float(s))


def green_P(m, kappa, z, s=None):
    """P^m_lambda(z) of eq. (Legendre_hypergeometric), kappa = -lambda(lambda+1)."""
    z, s0 = _zs(z)
    return _load().orc_green_P(int(m), float(kappa), z, s0 if s is None else float(s))


def jblock_green(m, kappa, z1, z2):
    """J^m(z1, z2) of eq. (Jmatrix_efficient), order 1, C_l = 1/(kappa + l(l+1)) for all l."""
    z1, s1 = _zs(z1)
    z2, s2 = _zs(z2)
    J = np.zeros(1)
    _load().orc_jblock_green(int(m), float(kappa), z1, s1, z2, s2, _p(J))
    return float(J[0])


def jblock_green2(m, kappas, z1, z2):
    """J^m(z1, z2) of order 2 in the basis (g, U g) from the Green's functions of two distinct
    kappa (eqs. (C_ell_efficient), (Jmatrix_efficient)), C_l = 1/((kappa_1 + l(l+1))(kappa_2 + l(l+1)))
    for every l; a 2 x 2 array."""
    z1, s1 = _zs(z1)
    z2, s2 = _zs(z2)
    k = np.ascontiguousarray(kappas, dtype=np.float64)
    J = np.zeros(4)
    _load().orc_jblock_green2(int(m), _p(k), z1, s1, z2, s2, _p(J))
    return J.reshape(2, 2)


def setup_green2(kappas, n_theta, n_phi, sets=None, modes=None, z=None):
    """Alg. 1 at order 2 in the basis (g, U g) on the Green's-function cross covariances of two
    distinct kappa (no band limit; modes m <= n_phi/2 - 1, or the listed ones).  Returns
    (A, B), each [sets][modes][2][2]."""
    mt = n_phi // 2 - 1
    md = np.arange(mt + 1, dtype=np.int32) if modes is None else np.ascontiguousarray(modes, dtype=np.int32)
    ns = n_sets(n_theta) if sets is None else min(sets, n_sets(n_theta))
    A = np.zeros((ns, len(md), 2, 2))
    B = np.zeros((ns, len(md), 2, 2))
    kap = np.ascontiguousarray(kappas, dtype=np.float64)
    zg = _zgrid(z, n_theta)
    rc = _load().orc_setup_modes_zb(2, 3, 0, _p(kap), n_theta, None if zg is None else _p(zg), ns,
                                    md.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(md), _p(A), _p(B))
    if rc != 0:
        raise ValueError("orc_setup_modes_zb rejected its arguments")
    return A, B


def greenc_G(m, kappa, x):
    """G_m(x) = 2F1(-lambda, lambda+1; 1+m; (1-x)/2) for complex kappa = -lambda(lambda+1)."""
    x, s = _zs(x)
    out = np.zeros(2)
    _load().orc_greenc_G(int(m), float(np.real(kappa)), float(np.imag(kappa)), x, s, _p(out))
    return complex(out[0], out[1])


def jblock_green2c(m, alpha, beta, z1, z2):
    """J^m(z1, z2) of order 2 in the basis (g, U g) from the Green's functions of the complex
    pair kappa = alpha +- i beta (C_l = 1/((l(l+1) + alpha)^2 + beta^2)); a 2 x 2 array."""
    z1, s1 = _zs(z1)
    z2, s2 = _zs(z2)
    k = np.array([alpha, beta], dtype=np.float64)
    J = np.zeros(4)
    _load().orc_jblock_green2c(int(m), _p(k), z1, s1, z2, s2, _p(J))
    return J.reshape(2, 2)


def setup_green2c(alpha, beta, n_theta, n_phi, sets=None, modes=None, z=None):
    """Alg. 1 at order 2 in the basis (g, U g) on the Green's-function cross covariances of the
    pair alpha +- i beta (no band limit; modes m <= n_phi/2 - 1, or the listed ones)."""
    mt = n_phi // 2 - 1
    md = np.arange(mt + 1, dtype=np.int32) if modes is None else np.ascontiguousarray(modes, dtype=np.int32)
    ns = n_sets(n_theta) if sets is None else min(sets, n_sets(n_theta))
    A = np.zeros((ns, len(md), 2, 2))
    B = np.zeros((ns, len(md), 2, 2))
    kap = np.array([alpha, beta], dtype=np.float64)
    zg = _zgrid(z, n_theta)
    rc = _load().orc_setup_modes_zb(2, 4, 0, _p(kap), n_theta, None if zg is None else _p(zg), ns,
                                    md.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(md), _p(A), _p(B))
    if rc != 0:
        raise ValueError("oracle setup_green2c failed")
    return A, B


def setup_green(kappa, n_theta, n_phi, sets=None, modes=None, z=None):
    """Alg. 1 at order 1 on the Green's-function cross covariances of Sec. 3 (C_l =
    1/(kappa + l(l+1)) for every l, no band limit; modes m <= n_phi/2 - 1, or the listed
    ones).  Returns (A, B), each [sets][modes][1][1]."""
    mt = n_phi // 2 - 1
    md = np.arange(mt + 1, dtype=np.int32) if modes is None else np.ascontiguousarray(modes, dtype=np.int32)
    ns = n_sets(n_theta) if sets is None else min(sets, n_sets(n_theta))
    A = np.zeros((ns, len(md), 1, 1))
    B = np.zeros((ns, len(md), 1, 1))
    kap = np.array([float(kappa)])
    zg = _zgrid(z, n_theta)
    rc = _load().orc_setup_modes_zb(1, 2, 0, _p(kap), n_theta, None if zg is None else _p(zg), ns,
                                    md.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(md), _p(A), _p(B))
    if rc != 0:
        raise ValueError("orc_setup_modes_zb rejected its arguments")
    return A, B


def ring_zs(n_theta, i):
    """(z_i, sin theta_i) of ring i, through the complementary angle (exact at the equator)."""
    z = ctypes.c_double()
    s = ctypes.c_double()
    _load().orc_ring_zs(n_theta, i, ctypes.byref(z), ctypes.byref(s))
    return z.value, s.value


def jblock_ring(order, m, ell_max, C, n_theta, i1, i2):
    """J^m(z_{i1}, z_{i2}) at two rings of the grid (ring values as the setup uses them)."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    z1, s1 = ring_zs(n_theta, i1)
    z2, s2 = ring_zs(n_theta, i2)
    J = np.zeros(order * order)
    _load().orc_jblock_zs(order, m, ell_max, _p(C), z1, s1, z2, s2, _p(J))
    return J.reshape(order, order)


def n_sets(n_theta):
    return _load().orc_n_sets(n_theta)


def start_ring(n_theta):
    return _load().orc_start_ring(n_theta)


def m_top(ell_max, n_phi):
    return _load().orc_m_top(ell_max, n_phi)


def _zgrid(z, n_theta):
    if z is None:
        return None
    z = np.ascontiguousarray(z, dtype=np.float64)
    if z.shape != (n_theta,):
        raise ValueError("z must hold n_theta ring values")
    return z


def setup(order, C, n_theta, n_phi, sets=None, z=None, basis="z"):
    """Alg. 1.  Returns (A, B), each [sets][m_top+1][order][order]; set 0 holds B_eq.
    z: optional ring values (north to south, symmetric about the equator); default the
    ring centres.  basis: "z" (value and z-derivatives) or "u" (order 2: (g, U g), Sec. 3)."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    ell_max = len(C) - 1
    mt = m_top(ell_max, n_phi)
    ns = n_sets(n_theta) if sets is None else min(sets, n_sets(n_theta))
    A = np.zeros((ns, mt + 1, order, order))
    B = np.zeros((ns, mt + 1, order, order))
    zg = _zgrid(z, n_theta)
    if basis == "z":
        rc = _load().orc_setup_z(order, ell_max, _p(C), n_theta, None if zg is None else _p(zg), n_phi, ns,
                                 _p(A), _p(B))
    else:
        md = np.arange(mt + 1, dtype=np.int32)
        rc = _load().orc_setup_modes_zb(order, {"u": 1}[basis], ell_max, _p(C), n_theta,
                                        None if zg is None else _p(zg), ns,
                                        md.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(md), _p(A), _p(B))
    if rc != 0:
        raise ValueError("orc_setup rejected its arguments")
    return A, B


def jblock_u(m, ell_max, C, z1, z2):
    """J^m(z1, z2) of order 2 in the basis (g, U g) of Sec. 3 (U L_lm through L_{l,m+1})."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    s1 = math.sqrt((1.0 - z1) * (1.0 + z1))
    s2 = math.sqrt((1.0 - z2) * (1.0 + z2))
    J = np.zeros(4)
    _load().orc_jblock_zs_u(m, ell_max, _p(C), float(z1), s1, float(z2), s2, _p(J))
    return J.reshape(2, 2)


def setup_modes(order, C, n_theta, modes, sets=None, z=None):
    """Alg. 1 for the listed modes only: (A, B), each [sets][len(modes)][order][order]."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    md = np.ascontiguousarray(modes, dtype=np.int32)
    ns = n_sets(n_theta) if sets is None else min(sets, n_sets(n_theta))
    A = np.zeros((ns, len(md), order, order))
    B = np.zeros((ns, len(md), order, order))
    zg = _zgrid(z, n_theta)
    rc = _load().orc_setup_modes_z(order, len(C) - 1, _p(C), n_theta, None if zg is None else _p(zg), ns,
                                   md.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(md), _p(A), _p(B))
    if rc != 0:
        raise ValueError("orc_setup_modes rejected its arguments")
    return A, B


def setup_asym(order, C, n_theta, n_phi, z, modes=None, basis="z"):
    """Alg. 1 on any strictly decreasing grid z (north to south, not necessarily symmetric):
    (A, B) for the northern walk and (As, Bs) for the southern walk in its own (true)
    coordinates, each [sets][modes][order][order]; default every mode m = 0..m_top.  basis
    as in setup."""
    C = np.ascontiguousarray(C, dtype=np.float64)
    ell_max = len(C) - 1
    md = np.arange(m_top(ell_max, n_phi) + 1, dtype=np.int32) if modes is None else \
        np.ascontiguousarray(modes, dtype=np.int32)
    ns = n_sets(n_theta)
    zg = _zgrid(z, n_theta)
    out = [np.zeros((ns, len(md), order, order)) for _ in range(4)]
    rc = _load().orc_setup_modes_asym_b(order, {"z": 0, "u": 1}[basis], ell_max, _p(C), n_theta, _p(zg), ns,
                                        md.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(md),
                                        *[_p(a) for a in out])
    if rc != 0:
        raise ValueError("orc_setup_modes_asym rejected its arguments")
    return tuple(out)


def sample_modes_list(order, n_theta, modes, A, B, seed, count, sets=None, south=None):
    """Chains of the listed modes: g[count][n_theta][len(modes)] complex (NaN where unreached).
    south: (As, Bs), the southern walk's own sets in true coordinates (default: the mirror of
    the northern sets)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    md = np.ascontiguousarray(modes, dtype=np.int32)
    ns = A.shape[0] if sets is None else sets
    g = np.empty((count, n_theta, len(md), 2))
    if south is None:
        _load().orc_sample_modes_list(order, n_theta, md.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                      len(md), ns, _p(A), _p(B), int(seed), count, _p(g))
    else:
        As = np.ascontiguousarray(south[0], dtype=np.float64)
        Bs = np.ascontiguousarray(south[1], dtype=np.float64)
        _load().orc_sample_modes_list_south(order, n_theta, md.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                            len(md), ns, _p(A), _p(B), _p(As), _p(Bs), int(seed), count, _p(g))
    return g[..., 0] + 1j * g[..., 1]


def max_threads():
    """OpenMP threads the oracle's parallel loops use."""
    return _load().orc_max_threads()


def set_threads(n):
    """Sets the OpenMP threads of the oracle's parallel loops (results do not depend on it)."""
    _load().orc_set_threads(int(n))


def philox(ctr, key):
    """Philox4x32-10 block for a 4-word counter and a 2-word key."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    _load().orc_philox(c, k, o)
    return [int(x) for x in o]


def normal(key, m, part, ring, order, q):
    """xi_q that produces ring `ring` of chain (m, part) for the field keyed `key`."""
    return _load().orc_normal(int(key), m, part, ring, order, q)


def sample_modes(order, n_theta, A, B, seed, count, sets=None):
    """Alg. 2 chains: g[count][n_theta][m_top+1] complex (NaN where no factor set reaches)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    ns = A.shape[0] if sets is None else sets
    mt = A.shape[1] - 1
    g = np.empty((count, n_theta, mt + 1, 2))
    _load().orc_sample_modes(order, n_theta, mt, ns, _p(A), _p(B), int(seed), count, _p(g))
    return g[..., 0] + 1j * g[..., 1]


def dft(g, n_phi, r0=0, r1=None):
    """Alg. 2 last step on rings [r0, r1): T[count][r1-r0][n_phi] (unnormalised C2R)."""
    count, n_theta, mt1 = g.shape
    r1 = n_theta if r1 is None else r1
    gi = np.empty((count, n_theta, mt1, 2))
    gi[..., 0] = g.real
    gi[..., 1] = g.imag
    T = np.empty((count, r1 - r0, n_phi))
    _load().orc_dft(n_theta, n_phi, mt1 - 1, count, r0, r1, _p(gi), _p(T))
    return T


def ring_offsets(n_ring):
    """Start of each ring in a field of rings with n_ring[i] pixels each (length n + 1)."""
    return np.concatenate([[0], np.cumsum(np.asarray(n_ring, dtype=np.int64))])


def dft_rings(g, n_ring, phi0):
    """Alg. 2 last step on rings with their own pixel counts n_ring[i] and first-pixel
    longitudes phi0[i]: T[count][sum n_ring], ring i at ring_offsets(n_ring)[i].  Every mode
    of g is kept (those above n_ring[i] / 2 alias onto the ring's pixels)."""
    count, n_theta, mt1 = g.shape
    nr = np.ascontiguousarray(n_ring, dtype=np.int32)
    p0 = np.ascontiguousarray(phi0, dtype=np.float64)
    off = ring_offsets(nr)
    assert nr.shape == (n_theta,) and p0.shape == (n_theta,) and np.all(nr >= 1)
    gi = np.empty((count, n_theta, mt1, 2))
    gi[..., 0] = g.real
    gi[..., 1] = g.imag
    T = np.empty((count, int(off[-1])))
    rc = _load().orc_dft_rings(n_theta, mt1 - 1, count, nr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(p0),
                               off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(gi), _p(T))
    assert rc == 0
    return T


def sample(order, n_theta, n_phi, A, B, seed, count, south=None):
    """Full plain method (chains + DFT), returns (T, g).  south: as in sample_modes_list."""
    if south is None:
        g = sample_modes(order, n_theta, A, B, seed, count)
    else:
        g = sample_modes_list(order, n_theta, np.arange(A.shape[1]), A, B, seed, count, south=south)
    return dft(g, n_phi), g
