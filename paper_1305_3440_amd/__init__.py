"""MI355X-native (gfx950) lattice Landau gauge fixing: checkerboard SU(3)
overrelaxation / stochastic relaxation sweeps behind the C ABI of
include/lgf.h.  The Python side is a ctypes binding of that ABI."""
from .lgf import *  # noqa: F401,F403
from .lgf import Ensemble, Lattice, LgfError, load_library  # noqa: F401

__all__ = [name for name in dir() if name.startswith(("lgf_", "LGF_"))] + [
    "Ensemble", "Lattice", "LgfError", "load_library"]
