"""MI355X (gfx950) implementation of the coupled density / total-energy D2Q9
MRT lattice Boltzmann step of Huang, Wu & Adams (arXiv:1809.08683).

The compute path is the HIP library ``liblbm_hip.so`` (C ABI in
``include/lbm.h``); ``lbm`` is its ctypes binding, ``inputs`` holds seeded
problem presets, ``build`` compiles the library for gfx950.
"""
__all__ = ["lbm", "inputs", "build"]
