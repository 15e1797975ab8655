"""MI355X-native implicit MPM step of HOT (Hierarchical Optimization Time
Integration, arXiv 1911.07913): HIP kernels behind the C ABI of include/hot.h,
with a thin ctypes binding in ``hot``."""
from . import hot  # noqa: F401
from .hot import Scene, Batch, HOT_FP64, HOT_MIXED  # noqa: F401
