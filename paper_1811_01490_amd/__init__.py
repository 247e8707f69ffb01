"""MI355X (gfx950) library for FFT and polynomial multiplication over Z/pZ,
p = r^k + 1 a Generalized Fermat prime (arXiv:1811.01490).  The compute path
is the HIP library libgfpfft.so (C ABI in include/gfp.h); ``gfp`` is its
Python binding."""

from .gfp import (GFP_EAGAIN, GFP_ECANCELED, GFP_ENOMEM, GFP_OK, Field, GFPError, Server, lib,  # noqa: F401
                  to_device, to_host)
