"""Rendering constants the paper leaves unstated (it defers to "standard 3DGS").

Each value is a reading of the paper; the oracle and the kernels receive the same
numbers at run time, so a different reading changes inputs, not code.
"""
from dataclasses import dataclass, field


@dataclass
class RenderSettings:
    alpha_min: float = 1.0 / 255.0   # a Gaussian with alpha below this is skipped
    alpha_max: float = 0.99          # alpha is clamped to at most this
    t_min: float = 1e-4              # compositing stops before transmittance drops below this
    blur: float = 0.3                # px^2 added to the diagonal of the 2D covariance
    z_near: float = 0.2              # Gaussians with camera depth below this are culled
    fov_clamp: float = 1.3           # x/z, y/z clamped to +-1.3 half-FOV tangents inside J
    bg: tuple = field(default_factory=lambda: (0.0, 0.0, 0.0))
    tile: int = 16                   # tile edge in pixels (binning only; results do not depend on it)
