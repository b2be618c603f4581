"""Enforced-sparsity NMF (alternating least squares with per-column top-t
sparsity) on AMD MI355X: a HIP library behind a C ABI plus its Python
binding.  See include/nmf.h for the ABI."""

from .nmf import (  # noqa: F401
    NMF,
    NMFError,
    NMFLoss,
    load_library,
    nmf_config,
    nmf_als_step,
    nmf_create,
    nmf_destroy,
    nmf_error,
    nmf_get_factors,
    nmf_get_pre,
    nmf_get_sparse,
    nmf_half_step,
    nmf_history,
    nmf_last_error,
    nmf_loss_bwd,
    nmf_loss_fwd,
    nmf_max_nnz,
    nmf_residual,
    nmf_set_factors,
    nmf_workspace_size,
    NMF_MODE_COLUMN,
    NMF_MODE_NONE,
    NMF_MODE_WHOLE,
    NMF_F32,
    NMF_F64,
    NMF_FLAG_NO_METRICS,
)
