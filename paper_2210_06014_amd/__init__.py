"""MI355X-native FasterTucker hot path (arXiv 2210.06014).

The arithmetic runs in hand-written HIP kernels inside libfastertucker.so,
reached through the C-ABI of include/fastertucker.h.  This package only
marshals arguments: PyTorch supplies device memory and the current stream.
"""
from ._lib import FT_KEEP_HOST, FT_WITH_PERM, FtError, SYMBOLS, load  # noqa: F401
from .api import (  # noqa: F401
    Params,
    Plan,
    core_epoch,
    core_grad,
    core_pass,
    epoch,
    factor_epoch,
    factor_pass,
    forward,
    grad,
    loss,
    loss_noalloc,
    predict,
    refresh,
    supported,
)
from .autograd import Reconstruction, reconstruct  # noqa: F401,E402
