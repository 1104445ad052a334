"""MI355X (gfx950) implementation of the RSA-exponentiation pseudorandom generator of
Datephanyawat & Beale (arXiv:1811.11629): HIP kernels behind the C ABI in
include/rsaprng.h, with a thin ctypes binding in :mod:`.rsaprng`."""
from . import rsaprng  # noqa: F401

__all__ = ["rsaprng"]
