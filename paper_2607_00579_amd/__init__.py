"""MI355X-native (gfx950) hot path of EPO's edge-based pose optimization.

The work is done by hand-written HIP kernels behind the C-ABI library
`libepo.so` (declared in include/epo.h).  This package holds the thin Python
binding (`_lib`), the plan object and the autograd wrapper (`api`), and the
plain torch-autograd comparison form (`autograd_baseline`).
"""
__version__ = "0.1.0"
