"""MI355X-native HyRes hyperspectral denoiser (HIP kernels for gfx950 behind a C ABI).

The public Python surface is in :mod:`paper_2204_06979_amd.api`; the seeded
workload generator is :mod:`paper_2204_06979_amd.synth`.
"""
__all__ = ["api", "synth"]
