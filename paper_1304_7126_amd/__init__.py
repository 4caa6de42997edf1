"""MI355X-native explicit M1 radiative-transfer step (Rosdahl et al. 2013).

The compute path is librtm1.so (hand-written HIP kernels for gfx950 behind
the C ABI of include/rtm1.h).  This package holds its build script, the
ctypes declarations (capi) and a torch-backed driver (runtime) that only
marshals arguments; torch supplies device memory and the stream.
"""
from . import capi  # noqa: F401

__all__ = ["capi", "RTContext", "group_attributes", "hll_table"]


def __getattr__(name):
    if name in ("RTContext", "group_attributes", "hll_table", "spectrum_attributes"):
        from . import runtime
        return getattr(runtime, name)
    raise AttributeError(name)
