"""MI355X-native TR-BDF2 / DG incompressible Navier-Stokes hot path.

The computation lives in the HIP library ``libtrbdg.so`` (sources in
``csrc/``, C interface in ``include/trbdg.h``); ``trbdg`` is its thin ctypes
binding.
"""
from .trbdg import (Adaptive, Context, Net, TrbdgError, load_library, solver_opts, EXPORTED, LIB_PATH)

__all__ = ["Adaptive", "Context", "Net", "TrbdgError", "load_library", "solver_opts", "EXPORTED", "LIB_PATH"]
