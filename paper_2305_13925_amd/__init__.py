"""MI355X-native Jac-PCG RZF precoder.

The compute path is libjacpcg.so (hand-written gfx950 HIP kernels behind a C
ABI, include/jacpcg.h); ``binding`` is its ctypes binding with the same names.
"""

from .binding import (  # noqa: F401
    Session,
    JacpcgError,
    jacpcg_gram,
    jacpcg_solve,
    rzf_precoder,
    rzf_precoder_plain,
    jacpcg_submit,
    jacpcg_poll,
    jacpcg_wait,
    jacpcg_cancel,
    jacpcg_session_clock_us,
    lib,
    status_string,
    last_error,
    GRAM_FP32,
    GRAM_BF16X3,
    GRAM_BF16X6,
    REFINE_FP64,
    PRECOND_JACOBI,
    PRECOND_NONE,
    EPILOGUE_FP32,
)
