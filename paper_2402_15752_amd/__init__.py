"""MI355X coupled phase-field lattice Boltzmann step (arXiv 2402.15752).

The hot path lives in ``libcplb.so`` (hand-written HIP for gfx950, C-ABI in
``include/cplb.h``); ``cplb`` is its ctypes binding.
"""
from . import cplb  # noqa: F401
from .cplb import Lattice, CplbError  # noqa: F401

__all__ = ["cplb", "Lattice", "CplbError"]
