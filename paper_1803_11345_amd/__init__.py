"""MI355X (gfx950) implementation of the hybrid central-moments / BGK lattice Boltzmann step for
the coupled Cahn-Hilliard--Navier-Stokes equations (De Rosis, Saito, Kaneko, Abe,
arXiv:1803.11345).

The compute path is liblbcm.so (HIP, see csrc/lbcm.hip and include/lbcm.h); ``lbcm`` is its
ctypes binding (the library itself is loaded on first use) and ``inputs`` builds the seeded
synthetic initial states.
"""
from . import inputs, lbcm  # noqa: F401

__all__ = ["inputs", "lbcm"]
