"""MI355X-native hybrid spectral deferred correction (HSDC) and two-level PFASST
for the monodomain equation (arXiv 2405.19994).

The compute path is the HIP library csrc/ -> libhsdc.so (C ABI: include/hsdc.h);
`hsdc` is its thin Python binding.
"""
from . import hsdc  # noqa: F401
