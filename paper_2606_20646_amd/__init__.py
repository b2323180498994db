"""MI355X (gfx950) implementation of the total-Lagrangian vectorial lattice
Boltzmann method for finite-strain hyperelasticity with curved boundaries.

The compute path is the HIP library ``libtlvlbm.so`` behind the C ABI in
``include/tlvlbm.h``; ``tlvlbm.Solver`` is its thin Python binding.
"""
from .tlvlbm import (DIRICHLET, FP32, FP64, NEUMANN, LIB_PATH, Solver,  # noqa: F401
                     TlvlbmError)
