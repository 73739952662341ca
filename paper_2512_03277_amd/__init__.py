"""MI355X-native batched SCC-DFTB + multimode cavity molecular dynamics.

The compute path is libcavdftb.so (hand-written HIP kernels for gfx950, C ABI
declared in include/cavdftb.h); `binding` is its thin ctypes wrapper.  There is
no CPU fallback: using the binding without the built library raises.
"""
from .binding import (EIG_AUTO, EIG_FULL, EIG_JACOBI, BORN_FD, BORN_FD_FORWARD, BORN_FIELD, BORN_MULLIKEN, BORN_SURROGATE, N_OBS, OBS_NAMES, SG_MEMBERS, SG_N_IN, SG_N_NORM,
                      SG_N_OUT, SG_N_PARAM, WORK_CHARGES, WORK_DIPOLE, WORK_ENERGY, WORK_FIELD, WORK_FORCES,
                      WORK_MU_POL, CavdftbError, Context, context_from_system, load_library, LIB_PATH, SYMBOLS)

__all__ = ["EIG_AUTO", "EIG_FULL", "EIG_JACOBI", "BORN_FD", "BORN_FD_FORWARD", "BORN_FIELD", "BORN_MULLIKEN", "BORN_SURROGATE", "N_OBS", "OBS_NAMES", "SG_MEMBERS", "SG_N_IN",
           "SG_N_NORM", "SG_N_OUT", "SG_N_PARAM", "CavdftbError", "Context", "context_from_system", "load_library",
           "LIB_PATH", "SYMBOLS", "WORK_CHARGES", "WORK_DIPOLE", "WORK_ENERGY", "WORK_FIELD", "WORK_FORCES",
           "WORK_MU_POL"]
