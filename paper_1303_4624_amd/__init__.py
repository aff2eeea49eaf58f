"""MI355X-native thermal lattice Boltzmann hot path (D2Q33 / D3Q95 on-lattice
models, 4th-order Hermite equilibrium, BGK), built as the HIP library
liblbm.so with a C ABI (include/lbm.h) and this thin Python binding.

    from paper_1303_4624_amd import Simulation, LBMFunction
    from paper_1303_4624_amd import _lib   # the C-ABI functions by name

The library must be built first (``python -m paper_1303_4624_amd.build``);
calls fail with RuntimeError otherwise.
"""
from . import _lib
from ._lib import LBMError, library

__all__ = ["_lib", "LBMError", "library", "Simulation", "LBMFunction"]


def __getattr__(name):
    # torch-dependent pieces are imported on first use
    if name == "Simulation":
        from .sim import Simulation
        return Simulation
    if name == "LBMFunction":
        from .autograd import LBMFunction
        return LBMFunction
    raise AttributeError(name)
