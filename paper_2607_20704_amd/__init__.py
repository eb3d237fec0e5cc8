"""MI355X (gfx950) per-level AMR hydrodynamics update after RAMSES-GPU.

librg.so (HIP kernels behind the C ABI in include/rg.h) does the work;
`api` is its thin PyTorch binding and `inputs` generates seeded workloads.
"""
__all__ = ["api", "inputs"]
