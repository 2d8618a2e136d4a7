"""MI355X-native matrix-free ILU(0) smoother (arXiv:2210.15280).

The compute lives in the HIP library libilu.so (C-ABI declared in
include/ilu.h).  This package only marshals arguments to it; PyTorch provides
device memory and streams.  Importing the package does not load the library;
`lib()` does, and raises if the library has not been built.
"""
from ._lib import (  # noqa: F401
    A_EXACT, A_SURROGATE, BOUNDARY_V1, BOUNDARY_V2, OVERLAP_FUSED, OVERLAP_OFF, OVERLAP_ON,
    COEFF_CONST, COEFF_EXPSINCOS, COEFF_POLY, COEFF_SINPROD, ILUError, SCHED_AUTO, SCHED_DATAFLOW, SCHED_PLANE,
    STORED_F64, STORED_SGS, SURR_F32, SURR_F64, Smoother, exported_symbols, header_symbols, lfa_orientation, lib,
    library_path, lfa_orientation_noalloc, LFA_NOALLOC_MAX_TETS,
)
