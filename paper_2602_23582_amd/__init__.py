"""MI355X-native random batch sum-of-Gaussians (RBSOG) force and pressure library.

The compute path is the C-ABI HIP library ``librbsog.so`` (declared in
``include/rbsog.h``); ``paper_2602_23582_amd.rbsog`` is its thin binding.
Importing this package loads nothing: the binding loads the library on first
use and raises if it is missing.
"""
__all__ = ["rbsog", "workloads"]
