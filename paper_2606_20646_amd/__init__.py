"""MI355X (gfx950) implementation of the total-Lagrangian vectorial lattice
Boltzmann method for finite-strain hyperelasticity with curved boundaries.

The compute path is the HIP library ``libtlvlbm.so`` behind the C ABI in
``include/tlvlbm.h``; ``tlvlbm.Solver`` is its thin Python binding.  The
binding (and with it the library) loads on first use of one of its names, so
that ``paper_2606_20646_amd.build`` can compile the library first.
"""
_EXPORTS = ("DIRICHLET", "FP32", "FP64", "NEUMANN", "LIB_PATH", "Solver", "TlvlbmError", "run_differentiable")


def __getattr__(name):
    if name in _EXPORTS:
        from . import tlvlbm
        return getattr(tlvlbm, name)
    raise AttributeError(name)
