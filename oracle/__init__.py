"""FP64 CPU oracle for the multi-view differentiable Gaussian-splat rasteriser.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or execute this
package: only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline` leg of `bench.py`
use it.  It shares no code with the HIP path (no kernels, headers, helpers, tables or
pre/post-processing); both consume the seeded inputs of `paper_2510_26358_amd.scenes`.

What it computes, and where the paper defines it (AgriGS-SLAM, arXiv 2510.26358):
  * Gaussian parameterisation (mean, covariance, opacity, SH colour)  -- Sec. III-B, the
    per-splat parameter equation; opacity as the sigmoid of a logit -- Sec. III-B,
    "Pruning" paragraph.
  * 3D covariance Sigma = R S S^T R^T                                 -- Sec. III-B.
  * image-space covariance Sigma' = J W Sigma W^T J^T, top-left 2x2   -- Sec. III-B.
  * front-to-back alpha compositing of colour / expected depth / alpha ("standard 3DGS",
    Sec. III-B, after Kerbl et al.), written as the per-pixel brute-force definition over
    all Gaussians: no tiles, no radius, no sort beyond the per-pixel depth order.
  * loss: the L1 part of L_3DGS and the LiDAR KL term L_LiDAR, summed -- Sec. III-C.
  * gradients to every Gaussian parameter and to each camera's SE(3) pose (poses refined
    by back-propagating through the projection -- abstract and Sec. III-C).
  * tile binning / key order as an integer reference (the kernel's float32 rect rule).
  * Adam on Gaussians and on se(3) pose increments, with an Exp retraction (the paper
    names no optimiser; this follows the refinement workload's stated setup).

Readings where the paper is silent (cutoffs, tile size, pixel centres, background, SH
convention, normalisations) are fixed in `RenderSettings`.

Parity status: every function here is pinned by the `-m "not gpu"` tests in
`tests/test_oracle_*.py` (closed forms, invariants, library special cases, Monte Carlo,
brute force, finite differences).  The paper prints no worked numeric example, so no
pin is a value quoted from it.
"""
from .settings import RenderSettings  # noqa: F401
