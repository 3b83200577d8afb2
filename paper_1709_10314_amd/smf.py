"""ctypes binding of libsmf (include/smf.h): the same entry points, argument marshalling only.

Device memory and streams come from PyTorch (``tensor.data_ptr()``,
``torch.cuda.current_stream().cuda_stream``); every step of setup and sampling runs in the
library's HIP kernels.  There is no fallback: if libsmf.so is missing or fails to load,
``load()`` raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmf.so")

SMF_OK, SMF_EINVAL, SMF_ENOMEM, SMF_EHIP, SMF_ENUMERIC = 0, -1, -2, -3, -4
SMF_FP64, SMF_FP32, SMF_NO_MIRROR, SMF_FUSED, SMF_UBASIS, SMF_GREEN, SMF_KAPPA_PAIR = 1, 2, 4, 8, 16, 32, 64

# every symbol include/smf.h declares
EXPORTS = ("smf_setup", "smf_setup_grid", "smf_sample", "smf_sample_lognormal", "smf_sample_modes", "smf_transform", "smf_set_ring_blocks",
           "smf_get_ring_blocks",
           "smf_plan_dims", "smf_get_factors", "smf_set_factors", "smf_plan_grid",
           "smf_destroy", "smf_error_string", "smf_setup_batch", "smf_batch_layout",
           "smf_sample_batch", "smf_sample_batch_packed", "smf_autotune_batch", "smf_setup_rings", "smf_ring_layout",
           "smf_synthesize_rings", "smf_sample_rings", "smf_sample_rings_lognormal", "smf_measure_normals",
           "smf_measure_fma", "smf_debug_fail_alloc", "smf_sample_rings_noalloc", "smf_set_log_level",
           "smf_batch_set_shape", "smf_batch_get_shape")


class smf_spectrum(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("n_kappa", ctypes.c_int),
                ("kappa", ctypes.POINTER(ctypes.c_double)),
                ("c_ell", ctypes.POINTER(ctypes.c_double)), ("ell_max", ctypes.c_int)]


class SmfError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {smf_error_string(code)} ({code})")


_lib = None


def load():
    """Load libsmf.so (built by paper_1709_10314_amd/build.py); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # PyTorch ships its own HIP runtime under the same soname; load it first so that the
    # library and torch's tensors and streams share one runtime in this process
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64
    lib.smf_setup.argtypes = [ctypes.POINTER(smf_spectrum), i, i, i, vp, ctypes.POINTER(vp)]
    lib.smf_setup_grid.argtypes = [ctypes.POINTER(smf_spectrum), i, ctypes.POINTER(ctypes.c_double), i, i, vp,
                                   ctypes.POINTER(vp)]
    lib.smf_sample.argtypes = [vp, u64, i, vp, vp]
    lib.smf_sample_lognormal.argtypes = [vp, u64, i, ctypes.c_double, ctypes.c_double, vp, vp]
    lib.smf_sample_modes.argtypes = [vp, u64, i, vp, vp]
    lib.smf_transform.argtypes = [vp, i, vp, vp]
    lib.smf_set_ring_blocks.argtypes = [vp, i]
    lib.smf_get_ring_blocks.argtypes = [vp, i, ctypes.POINTER(ctypes.c_int)]
    lib.smf_plan_dims.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
    lib.smf_get_factors.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.smf_set_factors.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), vp]
    lib.smf_plan_grid.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
    lib.smf_destroy.argtypes = [vp]
    lib.smf_error_string.argtypes = [i]
    lib.smf_error_string.restype = ctypes.c_char_p
    lib.smf_setup_batch.argtypes = [i, ctypes.POINTER(smf_spectrum), ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int), i, vp, ctypes.POINTER(vp)]
    lib.smf_batch_layout.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.smf_sample_batch.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(vp), vp]
    lib.smf_sample_batch_packed.argtypes = [vp, u64, vp, vp]
    lib.smf_autotune_batch.argtypes = [vp, u64, vp, vp, ctypes.POINTER(ctypes.c_int)]
    lib.smf_setup_rings.argtypes = [ctypes.POINTER(smf_spectrum), i, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double), i, vp,
                                    ctypes.POINTER(vp)]
    lib.smf_ring_layout.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.smf_synthesize_rings.argtypes = [vp, i, vp, vp, vp]
    lib.smf_sample_rings.argtypes = [vp, u64, i, vp, vp, vp]
    lib.smf_sample_rings_lognormal.argtypes = [vp, u64, i, ctypes.c_double, ctypes.c_double, vp, vp, vp]
    lib.smf_measure_normals.argtypes = [u64, i, i, vp, vp]
    lib.smf_measure_fma.argtypes = [i, i, vp, vp]
    lib.smf_debug_fail_alloc.argtypes = [i]
    lib.smf_sample_rings_noalloc.argtypes = [vp, u64, i, vp, vp]
    lib.smf_set_log_level.argtypes = [i]
    lib.smf_batch_set_shape.argtypes = [vp, i, i]
    lib.smf_batch_get_shape.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i)]
    for name in ("smf_setup", "smf_setup_grid", "smf_sample", "smf_sample_lognormal", "smf_sample_modes", "smf_transform", "smf_set_ring_blocks", "smf_get_ring_blocks",
                 "smf_plan_dims",
                 "smf_get_factors", "smf_set_factors", "smf_plan_grid", "smf_destroy", "smf_setup_batch", "smf_batch_layout",
                 "smf_sample_batch", "smf_sample_batch_packed", "smf_autotune_batch", "smf_setup_rings", "smf_ring_layout",
                 "smf_synthesize_rings", "smf_sample_rings", "smf_sample_rings_lognormal", "smf_measure_normals",
                 "smf_measure_fma", "smf_debug_fail_alloc", "smf_sample_rings_noalloc", "smf_set_log_level", "smf_batch_set_shape", "smf_batch_get_shape"):
        getattr(lib, name).restype = i
    _lib = lib
    return lib


def smf_error_string(code):
    return load().smf_error_string(int(code)).decode()


def _stream_handle(stream):
    if stream is None:
        import torch

        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _spectrum(order, ell_max, kappa, c_ell, keep):
    spec = smf_spectrum()
    spec.order = int(order)
    spec.ell_max = int(ell_max)
    if c_ell is not None:
        c = np.ascontiguousarray(c_ell, dtype=np.float64)
        keep.append(c)
        spec.c_ell = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        spec.n_kappa = 0
    else:
        k = np.ascontiguousarray([] if kappa is None else kappa, dtype=np.float64).reshape(-1)
        keep.append(k)
        spec.n_kappa = len(k)
        spec.kappa = k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if len(k) else None
    return spec


def smf_setup_rings(order, n_phi_ring, phi0, ell_max, kappa=None, c_ell=None, flags=SMF_FP32, stream=None,
                    z=None):
    """Returns (code, plan handle) of a ring plan: ring i with n_phi_ring[i] pixels from
    longitude phi0[i]; z as in smf_setup (None: ring centres)."""
    keep = []
    spec = _spectrum(order, ell_max, kappa, c_ell, keep)
    nr = np.ascontiguousarray(n_phi_ring, dtype=np.int32).reshape(-1)
    p0 = np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1)
    plan = ctypes.c_void_p()
    if len(p0) != len(nr) or (z is not None and len(z) != len(nr)):
        return SMF_EINVAL, plan
    zp = None
    if z is not None:
        zz = np.ascontiguousarray(z, dtype=np.float64).reshape(-1)
        keep.append(zz)
        zp = zz.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    rc = load().smf_setup_rings(ctypes.byref(spec), len(nr), zp, nr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                p0.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(flags),
                                _stream_handle(stream), ctypes.byref(plan))
    return rc, plan


def smf_ring_layout(plan, n_theta):
    off = (ctypes.c_int64 * (n_theta + 1))()
    rc = load().smf_ring_layout(plan, off)
    return rc, np.array([int(x) for x in off], dtype=np.int64)


def smf_synthesize_rings(plan, count, g_ptr, out_ptr, stream=None):
    return load().smf_synthesize_rings(plan, int(count), ctypes.c_void_p(g_ptr), ctypes.c_void_p(out_ptr),
                                       _stream_handle(stream))


def smf_sample_rings(plan, seed, count, g_ptr, out_ptr, stream=None):
    return load().smf_sample_rings(plan, ctypes.c_uint64(int(seed)), int(count), ctypes.c_void_p(g_ptr),
                                   ctypes.c_void_p(out_ptr), _stream_handle(stream))


def smf_sample_rings_noalloc(plan, seed, count, out_ptr, stream=None):
    return load().smf_sample_rings_noalloc(plan, ctypes.c_uint64(int(seed)), int(count), ctypes.c_void_p(out_ptr),
                                           _stream_handle(stream))


def smf_sample_rings_lognormal(plan, seed, count, mu, sigma, g_ptr, out_ptr, stream=None):
    return load().smf_sample_rings_lognormal(plan, ctypes.c_uint64(int(seed)), int(count), float(mu), float(sigma),
                                             ctypes.c_void_p(g_ptr), ctypes.c_void_p(out_ptr), _stream_handle(stream))


def smf_setup(order, n_theta, n_phi, ell_max, kappa=None, c_ell=None, flags=SMF_FP32, stream=None, z=None):
    """Returns (code, plan handle).  kappa: factors of C_l (eq. (Cl)); c_ell: explicit C_l;
    z: explicit ring values (north to south, symmetric; smf_setup_grid), default the ring
    centres (smf_setup)."""
    lib = load()
    spec = smf_spectrum()
    spec.order = int(order)
    spec.ell_max = int(ell_max)
    keep = []
    if c_ell is not None:
        c = np.ascontiguousarray(c_ell, dtype=np.float64)
        keep.append(c)
        spec.c_ell = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        spec.n_kappa = 0
    else:
        k = np.ascontiguousarray([] if kappa is None else kappa, dtype=np.float64).reshape(-1)
        keep.append(k)
        spec.n_kappa = len(k)
        spec.kappa = k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if len(k) else None
    plan = ctypes.c_void_p()
    if z is None:
        rc = lib.smf_setup(ctypes.byref(spec), int(n_theta), int(n_phi), int(flags),
                           _stream_handle(stream), ctypes.byref(plan))
    else:
        zz = np.ascontiguousarray(z, dtype=np.float64).reshape(-1)
        if len(zz) != int(n_theta):
            return SMF_EINVAL, plan
        keep.append(zz)
        rc = lib.smf_setup_grid(ctypes.byref(spec), int(n_theta), zz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                int(n_phi), int(flags), _stream_handle(stream), ctypes.byref(plan))
    return rc, plan


def smf_sample(plan, seed, count, out_ptr, stream=None):
    return load().smf_sample(plan, ctypes.c_uint64(int(seed)), int(count), ctypes.c_void_p(out_ptr),
                             _stream_handle(stream))


def smf_set_log_level(level):
    """Diagnostics level of the library (0 none, 1 setups and rejected arguments, 2 also each
    sampling call's launch shape; lines on stderr).  Returns the previous level."""
    return load().smf_set_log_level(int(level))


def smf_sample_lognormal(plan, seed, count, mu, sigma, out_ptr, stream=None):
    return load().smf_sample_lognormal(plan, ctypes.c_uint64(int(seed)), int(count), float(mu), float(sigma),
                                       ctypes.c_void_p(out_ptr), _stream_handle(stream))


def smf_sample_modes(plan, seed, count, g_ptr, stream=None):
    return load().smf_sample_modes(plan, ctypes.c_uint64(int(seed)), int(count), ctypes.c_void_p(g_ptr),
                                   _stream_handle(stream))


def smf_transform(plan, count, data_ptr, stream=None):
    return load().smf_transform(plan, int(count), ctypes.c_void_p(data_ptr), _stream_handle(stream))


def smf_set_ring_blocks(plan, blocks):
    return load().smf_set_ring_blocks(plan, int(blocks))


def smf_get_ring_blocks(plan, count):
    b = ctypes.c_int(0)
    rc = load().smf_get_ring_blocks(plan, int(count), ctypes.byref(b))
    return rc, b.value


def smf_plan_dims(plan):
    d = (ctypes.c_int * 8)()
    rc = load().smf_plan_dims(plan, d)
    return rc, list(d)


def smf_get_factors(plan, A, B):
    pd = ctypes.POINTER(ctypes.c_double)
    return load().smf_get_factors(plan, A.ctypes.data_as(pd), B.ctypes.data_as(pd))


def smf_plan_grid(plan, n_theta):
    """Returns (code, z values, symmetric flag)."""
    z = np.zeros(n_theta)
    sym = ctypes.c_int()
    rc = load().smf_plan_grid(plan, z.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(sym))
    return rc, z, bool(sym.value)


def smf_set_factors(plan, A, B, stream=None):
    pd = ctypes.POINTER(ctypes.c_double)
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    return load().smf_set_factors(plan, A.ctypes.data_as(pd), B.ctypes.data_as(pd), _stream_handle(stream))


def smf_destroy(plan):
    return load().smf_destroy(plan)


def _spectrum_struct(order, ell_max, kappa=None, c_ell=None, keep=None):
    spec = smf_spectrum()
    spec.order = int(order)
    spec.ell_max = int(ell_max)
    if c_ell is not None:
        c = np.ascontiguousarray(c_ell, dtype=np.float64)
        keep.append(c)
        spec.c_ell = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        spec.n_kappa = 0
    else:
        k = np.ascontiguousarray([] if kappa is None else kappa, dtype=np.float64).reshape(-1)
        keep.append(k)
        spec.n_kappa = len(k)
        spec.kappa = k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if len(k) else None
    return spec


def smf_setup_batch(fields, flags=SMF_FP32, stream=None):
    """fields: list of dicts with order, n_theta, n_phi, ell_max and kappa (list of kappa_i)
    or c_ell.  Returns (code, plan handle)."""
    keep = []
    n = len(fields)
    specs = (smf_spectrum * n)()
    nt = (ctypes.c_int * n)()
    npf = (ctypes.c_int * n)()
    for i, f in enumerate(fields):
        specs[i] = _spectrum_struct(f["order"], f["ell_max"], f.get("kappa"), f.get("c_ell"), keep)
        nt[i] = int(f["n_theta"])
        npf[i] = int(f["n_phi"])
    plan = ctypes.c_void_p()
    rc = load().smf_setup_batch(n, specs, nt, npf, int(flags), _stream_handle(stream), ctypes.byref(plan))
    return rc, plan


def smf_batch_layout(plan, n):
    off = (ctypes.c_int64 * (n + 1))()
    rc = load().smf_batch_layout(plan, off)
    return rc, [int(x) for x in off]


def smf_sample_batch(plan, seeds, out_ptrs, stream=None):
    """Field i drawn with key seeds[i] into the device buffer at out_ptrs[i]."""
    n = len(seeds)
    if len(out_ptrs) != n:
        raise ValueError("one output pointer per seed")
    sd = (ctypes.c_uint64 * n)(*[int(x) for x in seeds])
    op = (ctypes.c_void_p * n)(*[int(x) for x in out_ptrs])
    return load().smf_sample_batch(plan, sd, op, _stream_handle(stream))


def smf_sample_batch_packed(plan, seed, out_ptr, stream=None):
    return load().smf_sample_batch_packed(plan, ctypes.c_uint64(int(seed)), ctypes.c_void_p(out_ptr),
                                          _stream_handle(stream))


def smf_autotune_batch(plan, seed, out_ptr, stream=None):
    g = ctypes.c_int(0)
    rc = load().smf_autotune_batch(plan, ctypes.c_uint64(int(seed)), ctypes.c_void_p(out_ptr),
                                   _stream_handle(stream), ctypes.byref(g))
    return rc, g.value


class BatchPlan:
    """Many fields of uneven shape, spectrum and order, sampled by one call: a launch over
    every chain of every field, then one over every ring (a HIP graph can capture both)."""

    def __init__(self, fields, stream=None):
        rc, h = smf_setup_batch(fields, SMF_FP32, stream)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_setup_batch")
        self._h = h
        self.n = len(fields)
        self.fields = [dict(f) for f in fields]
        rc, self.offsets = smf_batch_layout(h, self.n)

    @property
    def handle(self):
        return self._h

    def empty(self, device="cuda"):
        import torch

        return torch.empty(self.offsets[-1], dtype=torch.float32, device=device)

    def sample(self, seed, out=None, stream=None):
        if out is None:
            out = self.empty()
        if not out.is_cuda or out.dtype.itemsize != 4 or out.numel() < self.offsets[-1]:
            raise ValueError("output must be a device float32 tensor of offsets[-1] elements")
        rc = smf_sample_batch_packed(self._h, seed, out.data_ptr(), stream)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_sample_batch_packed")
        return out

    def sample_fields(self, seeds, outs=None, stream=None):
        """Field i with key seeds[i] into its own tensor outs[i] ([n_theta, n_phi] float32 on
        the device; allocated when outs is None).  Returns the list of tensors."""
        import torch

        if len(seeds) != self.n:
            raise ValueError("one seed per field")
        if outs is None:
            outs = [torch.empty((f["n_theta"], f["n_phi"]), dtype=torch.float32, device="cuda")
                    for f in self.fields]
        for f, o in zip(self.fields, outs):
            if not o.is_cuda or o.dtype != torch.float32 or not o.is_contiguous() or \
                    o.numel() < f["n_theta"] * f["n_phi"]:
                raise ValueError("each output must be a contiguous device float32 tensor of n_theta * n_phi")
        rc = smf_sample_batch(self._h, seeds, [o.data_ptr() for o in outs], stream)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_sample_batch")
        return outs

    def field(self, out, i):
        """View of field i ([n_theta, n_phi]) in a packed output."""
        f = self.fields[i]
        return out[self.offsets[i]:self.offsets[i + 1]].view(f["n_theta"], f["n_phi"])

    def autotune(self, seed, out, stream=None):
        """Picks the launch shape (m-tiles per chain item, two launches or one persistent
        cooperative launch); returns the m-tile count."""
        rc, tiles = smf_autotune_batch(self._h, seed, out.data_ptr(), stream)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_autotune_batch")
        return tiles

    def set_shape(self, tiles, persistent):
        """tiles: m-tiles per chain item (1, 2, 4); persistent: one cooperative launch (True)
        or two launches (False) (smf_batch_set_shape)."""
        rc = load().smf_batch_set_shape(self._h, int(tiles), 1 if persistent else 0)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_batch_set_shape")

    def shape(self):
        """(tiles, persistent) of the plan (smf_batch_get_shape)."""
        t, p = ctypes.c_int(), ctypes.c_int()
        rc = load().smf_batch_get_shape(self._h, ctypes.byref(t), ctypes.byref(p))
        if rc != SMF_OK:
            raise SmfError(rc, "smf_batch_get_shape")
        return t.value, bool(p.value)

    def close(self):
        if getattr(self, "_h", None):
            smf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """A setup plan (Alg. 1 factors on the GPU) with sampling methods (Alg. 2)."""

    def __init__(self, order, n_theta, n_phi, ell_max, kappa=None, c_ell=None, precision="fp32",
                 stream=None, z=None, basis="z", mirror=True, green=False, kappa_pair=False):
        """basis: "z" (the state is the value and its z-derivatives) or "u" (order 2: (g, U g)
        of Sec. 3, SMF_UBASIS).  mirror=False stores the southern walk's own factor sets
        (SMF_NO_MIRROR).  green=True (order 1 with one kappa, order 2 with two distinct ones): the
        Green's-function setup of Sec. 3 for eq. (Cl) without band limit (SMF_GREEN; ell_max is
        ignored; at order 2 the state is (g, U g)).  kappa_pair=True with green at order 2:
        kappa = (alpha, beta) names the pair alpha +- i beta (SMF_KAPPA_PAIR)."""
        flags = {"fp32": SMF_FP32, "fp64": SMF_FP64}[precision] | {"z": 0, "u": SMF_UBASIS}[basis]
        if not mirror:
            flags |= SMF_NO_MIRROR
        if green:
            flags |= SMF_GREEN
        if kappa_pair:
            flags |= SMF_KAPPA_PAIR
        rc, h = smf_setup(order, n_theta, n_phi, ell_max, kappa=kappa, c_ell=c_ell, flags=flags,
                          stream=stream, z=z)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_setup" if z is None else "smf_setup_grid")
        self._adopt(h)

    def _adopt(self, h):
        self._h = h
        rc, d = smf_plan_dims(h)
        (self.order, self.n_theta, self.n_phi, self.ell_max, self.m_top, self.n_sets,
         self.start_ring, fl) = d
        self.precision = "fp64" if fl == SMF_FP64 else "fp32"
        rc, self.z, self.symmetric = smf_plan_grid(h, self.n_theta)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_plan_grid")

    @property
    def handle(self):
        return self._h

    def dtype(self):
        import torch

        return torch.float64 if self.precision == "fp64" else torch.float32

    def empty(self, count, device="cuda"):
        import torch

        return torch.empty((count, self.n_theta, self.n_phi), dtype=self.dtype(), device=device)

    def sample(self, seed, count, out=None, stream=None):
        """count fields keyed seed..seed+count-1 as a [count, n_theta, n_phi] tensor."""
        if out is None:
            out = self.empty(count)
        self._check_out(out, count)
        rc = smf_sample(self._h, seed, count, out.data_ptr(), stream)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_sample")
        return out

    def sample_lognormal(self, seed, count, mu=0.0, sigma=1.0, out=None, stream=None):
        """exp(mu + sigma T) of the fields sample(seed, count) would return."""
        if out is None:
            out = self.empty(count)
        self._check_out(out, count)
        rc = smf_sample_lognormal(self._h, seed, count, mu, sigma, out.data_ptr(), stream)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_sample_lognormal")
        return out

    def transform(self, data, count, stream=None):
        """In-place C2R of `count` fields of modes (the sample_modes layout) into fields;
        returns the [count, n_theta, n_phi] view of `data`."""
        self._check_out(data, count)
        rc = smf_transform(self._h, count, data.data_ptr(), stream)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_transform")
        return data.view(-1)[: count * self.n_theta * self.n_phi].view(count, self.n_theta, self.n_phi)

    def set_ring_blocks(self, blocks):
        """Affine-scan ring blocks: 0 automatic, 1 never, 2/4/8/16 always (capped)."""
        rc = smf_set_ring_blocks(self._h, blocks)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_set_ring_blocks")

    def ring_blocks(self, count):
        """Ring blocks a call with `count` fields uses (1 = plain recursion)."""
        rc, b = smf_get_ring_blocks(self._h, count)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_get_ring_blocks")
        return b

    def sample_modes(self, seed, count, out=None, stream=None):
        """Pre-FFT modes g_m as [count, n_theta, n_phi/2, 2] (Re, Im) in the sample dtype."""
        if out is None:
            out = self.empty(count)
        self._check_out(out, count)
        rc = smf_sample_modes(self._h, seed, count, out.data_ptr(), stream)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_sample_modes")
        return out.view(count, self.n_theta, self.n_phi // 2, 2)

    def _factor_shape(self):
        sets = self.n_sets * (1 if self.symmetric else 2)
        return (sets, self.m_top + 1, self.order, self.order)

    def factors(self):
        """FP64 (A, B), each [n_sets, m_top+1, order, order] (2 n_sets sets for a grid with no
        symmetry: the northern ones, then the southern walk's in true coordinates)."""
        shape = self._factor_shape()
        A = np.zeros(shape)
        B = np.zeros(shape)
        rc = smf_get_factors(self._h, A, B)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_get_factors")
        return A, B

    def set_factors(self, A, B, stream=None):
        """Replace the plan's factors with (A, B) of the factors() layout (Alg. 2's inputs)."""
        shape = self._factor_shape()
        if np.shape(A) != shape or np.shape(B) != shape:
            raise ValueError(f"factors must have shape {shape}")
        rc = smf_set_factors(self._h, A, B, stream)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_set_factors")

    def _check_out(self, out, count):
        if not out.is_cuda or out.dtype != self.dtype() or not out.is_contiguous():
            raise ValueError("output must be a contiguous device tensor of the plan's dtype")
        if out.numel() < count * self.n_theta * self.n_phi:
            raise ValueError("output tensor too small")

    def close(self):
        if getattr(self, "_h", None):
            smf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class RingPlan(Plan):
    """A plan on rings with their own pixel counts and first-pixel longitudes (iso-latitude
    grids such as HEALPix): every mode up to ell_max is sampled (the chains run at the
    power-of-two n_phi that keeps them all) and each ring is synthesised at its own pixels."""

    def __init__(self, order, n_phi_ring, phi0, ell_max, kappa=None, c_ell=None, precision="fp32",
                 stream=None, z=None, basis="z", green=False, kappa_pair=False):
        """green / kappa_pair: the Green's-function setup of Sec. 3 (as Plan) for the modes up
        to ell_max, which the rings are synthesised from."""
        flags = {"fp32": SMF_FP32, "fp64": SMF_FP64}[precision] | {"z": 0, "u": SMF_UBASIS}[basis]
        if green:
            flags |= SMF_GREEN
        if kappa_pair:
            flags |= SMF_KAPPA_PAIR
        rc, h = smf_setup_rings(order, n_phi_ring, phi0, ell_max, kappa=kappa, c_ell=c_ell, flags=flags,
                                stream=stream, z=z)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_setup_rings")
        self._adopt(h)
        self.n_phi_ring = np.asarray(n_phi_ring, dtype=np.int32).copy()
        self.phi0 = np.asarray(phi0, dtype=np.float64).copy()
        rc, self.offsets = smf_ring_layout(h, self.n_theta)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_ring_layout")
        self.pixels = int(self.offsets[-1])

    def empty_rings(self, count, device="cuda"):
        import torch

        return torch.empty((count, self.pixels), dtype=self.dtype(), device=device)

    def _check_rings(self, out, count):
        if not out.is_cuda or out.dtype != self.dtype() or not out.is_contiguous():
            raise ValueError("output must be a contiguous device tensor of the plan's dtype")
        if out.numel() < count * self.pixels:
            raise ValueError("output tensor too small")

    def sample_rings(self, seed, count, out=None, work=None, stream=None):
        """count fields keyed seed..seed+count-1 as a [count, pixels] tensor, ring i of a
        field at offsets[i]; work: a mode buffer as sample_modes takes (allocated if None)."""
        if out is None:
            out = self.empty_rings(count)
        if work is None:
            work = self.empty(count)
        self._check_rings(out, count)
        self._check_out(work, count)
        rc = smf_sample_rings(self._h, seed, count, work.data_ptr(), out.data_ptr(), stream)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_sample_rings")
        return out.view(-1)[: count * self.pixels].view(count, self.pixels)

    def sample_rings_noalloc(self, seed, count, out, stream=None):
        """sample_rings with no work buffer: the library's own device array holds the modes
        (smf_sample_rings_noalloc; at most 64 MiB of modes, calls on one device must not
        overlap).  `out` must be given: nothing is allocated."""
        self._check_rings(out, count)
        rc = smf_sample_rings_noalloc(self._h, seed, count, out.data_ptr(), stream)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_sample_rings_noalloc")
        return out.view(-1)[: count * self.pixels].view(count, self.pixels)

    def sample_rings_lognormal(self, seed, count, mu=0.0, sigma=1.0, out=None, work=None, stream=None):
        """exp(mu + sigma T) of the pixels sample_rings(seed, count) would return."""
        if out is None:
            out = self.empty_rings(count)
        if work is None:
            work = self.empty(count)
        self._check_rings(out, count)
        self._check_out(work, count)
        rc = smf_sample_rings_lognormal(self._h, seed, count, mu, sigma, work.data_ptr(), out.data_ptr(), stream)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_sample_rings_lognormal")
        return out.view(-1)[: count * self.pixels].view(count, self.pixels)

    def synthesize_rings(self, g, count, out=None, stream=None):
        """The rings of `count` fields of modes g (the sample_modes layout)."""
        if out is None:
            out = self.empty_rings(count)
        self._check_rings(out, count)
        self._check_out(g, count)
        rc = smf_synthesize_rings(self._h, count, g.data_ptr(), out.data_ptr(), stream)
        if rc != SMF_OK:
            raise SmfError(rc, "smf_synthesize_rings")
        return out.view(-1)[: count * self.pixels].view(count, self.pixels)
