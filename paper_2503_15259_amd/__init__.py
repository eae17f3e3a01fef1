"""MI355X-native PSCA device activity detection (arXiv 2503.15259).

The compute path is libpsca.so (HIP, gfx950) behind the C ABI in
include/psca.h; `psca` is its Python binding and `instances` the seeded
generator of synthetic detection instances.
"""
from . import instances  # noqa: F401

__all__ = ["instances", "psca"]


def __getattr__(name):
    if name == "psca":
        from . import psca as _p
        return _p
    raise AttributeError(name)
