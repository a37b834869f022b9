"""Ternary free-energy entropic lattice Boltzmann update on the MI355X.

A thin Python face of the C ABI in ``include/telbm.h`` (``libtelbm.so``,
HIP kernels for gfx950).  The method is that of Woehrwag, Semprebon,
Mazloomi, Karlin and Kusumaatmaja, "Ternary free-energy entropic lattice
Boltzmann model with high density ratio" (arXiv:1710.07486).
"""
from ._lib import D2Q9, D3Q27, FP64, FP32_MIXED, FIELDS, TelbmError  # noqa: F401
from .solver import (EOS_CS, EOS_PR, EOS_VDW, Params, Solver, coexistence, critical_temperature,  # noqa: F401
                     required_bytes, temperature_for_ratio)
from .nliquid import NLParams, NLSolver  # noqa: F401,E402
