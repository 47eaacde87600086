"""MI355X-native equivalent-charge ("replacement") fast multipole method
(Kajima, arXiv:2212.13080): HIP kernels for gfx950 behind a C ABI
(include/eqfmm.h), with a thin torch front end."""
from .native import (FP32, FP32_BF16FAR, FP64, FREE, FREE_CONTINUOUS, PERIODIC,  # noqa: F401
                     PERIODIC_CONTINUOUS, EqfmmError)
from .fmm import Plan, energy  # noqa: F401
