"""MI355X-native lattice Boltzmann intrinsic-permeability solver.

Submodules are imported on demand: ``qsgs`` (mask generator, host only) and
``lbm`` (the HIP solver behind the C ABI of ``include/lbm.h``).
"""
__all__ = ["qsgs", "lbm", "build"]
