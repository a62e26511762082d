"""MI355X-native multi-view differentiable Gaussian-splat rasteriser (AgriGS-SLAM hot path).

Importing the package loads nothing; the HIP library is loaded by `load()` or by the
first `Rasterizer`.  `scenes` holds the seeded synthetic inputs.
"""
from ._lib import load  # noqa: F401
