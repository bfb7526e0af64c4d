"""MI355X-native weighted-upwind vector kinetic lattice Boltzmann (WU-VKLB).

The hot path is the C-ABI library libvklb.so (HIP kernels for gfx950, see
include/vklb.h); `vklb` is its Python binding, `inputs` builds seeded initial
states for the workloads.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "vklb"]
