"""Exact per-camera covariance of bundle-adjusted reconstructions on MI355X.

The computation runs in the hand-written gfx950 HIP kernels of
``lib/libucov.so`` behind the C-ABI declared in ``include/ucov.h``; this
package is its thin Python binding (device memory and streams come from
torch).  See ``_binding.Context`` for the entry points.
"""
from ._binding import (BF16X_NS, FP32_NS, FP64, GAUGE_CAMERA, GAUGE_PAPER, Context, DeviceScene, UcovError,  # noqa: F401
                       EXPORTS, LIB_PATH, load)
