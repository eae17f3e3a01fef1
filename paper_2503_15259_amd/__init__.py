"""MI355X-native PSCA device activity detection (arXiv 2503.15259).

The compute path is libpsca.so (HIP, gfx950) behind the C ABI in
include/psca.h; `paper_2503_15259_amd.psca` is its Python binding and
`instances` the seeded generator of synthetic detection instances.
"""
from . import instances  # noqa: F401
