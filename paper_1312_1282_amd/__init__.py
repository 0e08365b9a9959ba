"""MI355X-native Jastrow variational Monte Carlo of liquid 4He.

The computation lives in libhevmc.so (HIP kernels for gfx950 behind the C ABI
of include/hevmc.h); ``abi`` binds it, ``configs`` holds the synthetic
workloads, ``observables`` the host post-processing of sampled quantities
(pair distribution, reweighting in b) and ``serving`` the request server.
"""
from . import configs  # noqa: F401

__all__ = ["abi", "configs"]
