"""MI355X-native convolutional gridding and degridding (gfx950 HIP kernels
behind a C ABI; PyTorch supplies device memory and streams).

    from paper_2508_17187_amd import lr
    cf = lr.lr_cf_build(grid_spec, cf_spec)
    lr.lr_grid(cf, vis, lr.LR_F32, grid)

Submodules: `lr` (the binding), `workload` (synthetic inputs to device
tensors), `autograd` (differentiable degridding), `serving` (continuous
batching of grid / degrid jobs).
"""

from . import lr  # noqa: F401
