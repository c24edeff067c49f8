"""MI355X-native hot path of SCSF (sorted Chebyshev-filtered subspace iteration).

The compute lives in libscsf.so (HIP for gfx950, C ABI declared in include/scsf.h);
`paper_2510_23215_amd.scsf` is the ctypes binding.
"""
from . import scsf  # noqa: F401
