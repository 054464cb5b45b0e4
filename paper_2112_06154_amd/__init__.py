"""MI355X (gfx950) distance-generalized (k,h)-core decomposition.

Exact (ExactCore) and sampled (Core, Alg. 4) (k,h)-cores and the densest core
level of Tatti, "Fast computation of distance-generalized cores using
sampling" (arXiv 2112.06154), computed by hand-written HIP kernels behind the
C ABI in include/khcore.h.  This package is only the Python binding.
"""
from .khcore import (Context, Graph, KhError, Server, buffer_size, core, core_batch, dense, hdeg,  # noqa: F401
                     hdeg_noalloc, ranks, sampled_lists, status_str, validate_csr)
from .khcore import (KH_EBUSY, KH_EDEVICE, KH_EGRAPH, KH_EINVAL, KH_ENOMEM, KH_ENOTFOUND,  # noqa: F401
                     KH_ENOTIMPL, KH_EOVERFLOW, KH_OK)
