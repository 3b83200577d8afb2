"""MI355X (gfx950) sampler of isotropic Gaussian random fields on the sphere.

Creasey & Lang, "Fast generation of isotropic Gaussian random fields on the sphere"
(arXiv:1709.10314): each azimuthal Fourier mode is a latitude-ring Gauss-Markov chain,
sampled outward from the equator, then an inverse FFT along phi gives the field.  The
work runs in the HIP library libsmf.so (C ABI in include/smf.h); ``smf`` is its binding.
"""
from . import smf  # noqa: F401
from .smf import BatchPlan, Plan, RingPlan, SmfError  # noqa: F401
