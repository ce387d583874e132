"""MI355X (gfx950) implementation of the checkerboard Metropolis sweep of the
2D Ising and Blume-Capel models and of the measurements taken while the
lattice relaxes after a quench (Bisson et al., arXiv:2502.18624).

The work runs in hand-written HIP kernels behind the C ABI of
``include/mcl.h`` (``libmcl.so``); this package marshals arguments and
supplies device memory and streams through PyTorch.
"""
from ._lib import (BC, CORR_FULL, CORR_NONE, CORR_PROTOCOL, INIT_DOWN, INIT_RANDOM,  # noqa: F401
                   INIT_UP, INIT_ZERO, ISING, ISING_LUT, MclError, lib)
from .lattice import (Lattice, correlation, correlation_length, energy, group_sweep, lut_table, query_bytes,  # noqa: F401
                      rset, schwinger_dyson, thresholds)
