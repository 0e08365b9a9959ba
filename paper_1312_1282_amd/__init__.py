"""MI355X-native Jastrow variational Monte Carlo of liquid 4He.

The computation lives in libhevmc.so (HIP kernels for gfx950 behind the C ABI
of include/hevmc.h); ``abi`` binds it, ``configs`` holds the synthetic
workloads and ``stats`` the post-processing of per-walker accumulators.
"""
from . import configs  # noqa: F401

__all__ = ["abi", "configs"]
