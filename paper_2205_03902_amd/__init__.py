"""Layer-wise inverse multislice ptychography (arXiv 2205.03902) on one MI355X.

The compute path is libimsp.so (HIP kernels for gfx950 behind the C ABI in
include/ms.h); this package holds its ctypes binding, the autograd wrapper,
the Algorithm 1 driver, workload geometries and the seeded input generator.
"""
__all__ = ["abi", "configs", "synth", "layerwise", "autograd"]
