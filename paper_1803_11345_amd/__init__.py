"""MI355X (gfx950) implementation of the hybrid central-moments / BGK lattice Boltzmann step for
the coupled Cahn-Hilliard--Navier-Stokes equations (De Rosis, Saito, Kaneko, Abe,
arXiv:1803.11345), with a learned convolutional surrogate of K steps of it.

The compute path is liblbcm.so (HIP, see csrc/lbcm.hip, csrc/surrogate.hip, include/lbcm.h and
include/lbcm_net.h); ``lbcm`` and ``net`` are its ctypes bindings (the library itself is loaded
on first use) and ``inputs`` builds the seeded synthetic initial states.
"""
from . import inputs, lbcm, net  # noqa: F401

__all__ = ["inputs", "lbcm", "net"]
