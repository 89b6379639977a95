"""MI355X (gfx950) library for randomized preconditioned Cholesky-QR.

Garrison & Ipsen, "A randomized preconditioned Cholesky-QR algorithm"
(arXiv 2406.11751).  The computation lives in HIP kernels behind the C ABI of
include/rpcholqr.h; this package only builds and binds that library.
"""
from .native import (FP64, FP32_REFINE, BF16X2_REFINE, A1_FP32, SMOOTH, BatchedPlan, RpCholQRError, colmajor_empty,  # noqa: F401
                     factor, factor_batched, factor_noalloc, load_batched_tuning, load_library, max_n,
                     precond_factor, sample_indices, set_batched_tuning, timing_enable, timing_read,
                     workspace_bytes)
