"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package draws scenes, rays and ragged sample batches with numpy and nothing
else.  It holds none of the rendering arithmetic (no interpolation, activation,
compositing, distortion or optimiser step): it only produces the FP32 buffers that
both the FP64 CPU oracle and the HIP path consume.
"""
from .scenes import (  # noqa: F401
    Grid, Rays, Samples, MLPWeights, Workload,
    blob_density, normal_grid, uniform_grid,
    rays_at_box, pinhole_rays, rays_into_ball, forward_facing_rays, slab_interval,
    uniform_samples, disparity_samples, mlp_weights, proposal_weights,
    config1, config2, config3, config4, config5, config6, random_ragged, proposal_rays,
)
