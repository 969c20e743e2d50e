"""MI355X (gfx950) MPS time stepper for the 1D1V Vlasov-Poisson equations
(Ye & Loureiro, arXiv:2205.11990).

The computation lives in the HIP library ``libmpsvlasov.so`` (C-ABI in
``include/mps_vlasov.h`` and ``include/mps_blocks.h``); ``binding`` is a thin
ctypes layer over it.  Importing this package does not load the library;
the first call does, and raises if it has not been built.
"""
from .binding import (MpsError, MpsState, add_compress, compress, gemm, lib,  # noqa: F401
                      operator, qr, set_jacobi_max_sweeps, stats, step_batched,
                      svd_truncate, workspace_bound)
