"""MI355X (gfx950) semantic Gaussian-splatting rasterizer: the differentiable
renderer of GS^3LAM (colour, depth, cumulative opacity and semantic features,
with gradients to every Gaussian parameter and to the camera pose).

Modules:
    build      compiles libsgs.so (HIP kernels + C ABI) in-tree
    _lib       ctypes binding of include/sgs.h (fails loudly if not built)
    raster     torch-facing driver, autograd wrapper, graph-friendly buffers
    batched    multi-view mapping step captured in a HIP graph
    autotune   tile / LDS-batch / launch-mode selection
    workloads  seeded synthetic inputs (no rasterizer arithmetic)
"""
__version__ = "1.0.0"
