"""MI355X (gfx950) B-ADMM Wasserstein barycenters and D2-clustering.

The compute path is the HIP library libd2.so (C ABI in include/d2.h);
`paper_1510_00012_amd.d2` is its thin ctypes binding.
"""
from .d2 import D2Context, D2Error, load_library  # noqa: F401
