"""MI355X-native lattice Boltzmann squirmers (arXiv:1903.04799).

The compute path is the gfx950 library ``liblbsq.so`` behind the C ABI of
``include/lbsq.h``; ``paper_1903_04799_amd.lbsq`` is its ctypes binding.
"""
from .lbsq import Sim, LBError, step_batch, load, strerror  # noqa: F401

__all__ = ["Sim", "LBError", "step_batch", "load", "strerror"]
