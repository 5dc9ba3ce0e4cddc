"""Multi-word (double-double / triple-double / quad-double) LU with partial
pivoting, substitutions and mixed-precision iterative refinement on one AMD
Instinct MI355X, after Kouya 2021 (arXiv 2107.12550), Sec. 2 and Listing 1.

Every step runs in the HIP kernels of ``libbnc.so`` behind the C-ABI of
``include/bnc.h``; this package only marshals arguments.  PyTorch provides
device memory and the current stream.
"""
from .bnc import (  # noqa: F401
    BNC_AUTO,
    BNC_BAD_SIZE,
    BNC_CONVERGED,
    BNC_ERR_HIP,
    BNC_ERR_TIMEOUT,
    BNC_ERR_UNSUPPORTED,
    BNC_ERR_WORKSPACE,
    BNC_MAX_ITER,
    BNC_NONFINITE,
    BNC_SINGULAR,
    BNC_STAGNATED,
    BNC_SPLIT_RANGE,
    BNC_TIMED_OUT,
    OP_ADD,
    OP_FMS,
    OP_MUL,
    OP_RECIP,
    OP_ROUND4,
    MLP,
    NFEATURES,
    BatchSolver,
    BncError,
    features,
    gemm,
    getrf,
    getrf_ozaki,
    getrf_workspace_size,
    getrs,
    getrs_workspace_size,
    lib,
    lib_path,
    mw_apply,
    oz_beta,
    profile_enable,
    profile_read,
    refine,
    refine_async,
    refine_result,
    refine_result_bytes,
    refine_workspace_size,
    residual,
    residual_workspace_size,
    test_force_timeout,
    wall_clock_khz,
)
