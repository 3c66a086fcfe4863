"""MI355X (gfx950) two-site ab initio DMRG sigma library.

The compute path is the HIP shared library ``libdmrg_mi355x.so`` behind the C
ABI of ``include/dmrg.h``; :mod:`._binding` is a thin ctypes binding of it.
"""
from ._binding import (Context, DMRGEnergy, DMRGError, load_library, validate, LIB_PATH, EXPORTS,  # noqa: F401
                       DMRG_FP64, DMRG_BF16, DMRG_BF16X3)
