"""MI355X (gfx950) fast direct solver for 2D quasi-periodic Dirichlet scattering.

The solver lives in the HIP library libqpscatter.so behind the C ABI of
include/qpscatter.h; ``binding`` is its thin Python binding (imported lazily so that
building and CPU-only tooling do not need the library), ``geometry`` discretizes curves.
"""
__all__ = ["binding", "geometry"]
