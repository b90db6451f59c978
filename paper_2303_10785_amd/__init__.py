"""MI355X-native gradient-based-reconstruction RHS (MEG6 + alpha-damping) on
curvilinear and moving grids: HIP kernels behind the C ABI of include/gbr.h,
with a thin ctypes binding (``gbr``)."""
from . import gbr  # noqa: F401
from .gbr import Grid, GbrError  # noqa: F401
