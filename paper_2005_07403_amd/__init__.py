"""MI355X-native batched 2x2 SVD (arXiv:2005.07403) and Kogbetliantz solver.

The compute path is libsvd2.so (hand-written HIP for gfx950) behind the C ABI
of include/svd2.h; this package holds its build script and a ctypes binding.
"""
from . import svd2  # noqa: F401
from .svd2 import (  # noqa: F401
    SVD2_BACKSCALE_ALL, SVD2_BACKSCALE_NONE, SVD2_BACKSCALE_SAFE, SVD2_RESCUE_FP64,
    SVD2_RESCUE_QUEUE, Svd2Error, csvd2_batch, dsvd2_batch, ssvd2_batch, svd2_workspace_bytes,
    zsvd2_batch,
)
