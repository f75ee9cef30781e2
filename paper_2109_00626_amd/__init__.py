"""Tensor contraction products on Tensor-Train cores for MI355X (gfx950).

All computation runs in libttc.so (hand-written HIP kernels behind a C ABI);
this package only marshals torch tensors into that ABI.  Importing fails if
the library has not been built."""
from .api import (  # noqa: F401
    BatchPlan,
    TTCError,
    tt_contract_inner,
    tt_contract_inner_bwd,
    tt_contract_inner_noalloc,
    tt_contract_modes,
    tt_contract_pairs,
    tt_contract_pairs_query,
    tt_contract_modes_query,
    tt_mode_n_product,
    tt_round,
    tt_svd,
    tt_svd_query,
    ttc_mse_loss,
    ttm_apply,
    ttm_apply_dense,
    ttm_apply_dense_bwd,
    ttm_apply_dense_query,
    version,
)
from .autograd import TTInner, TTLinear, tt_inner, tt_linear  # noqa: F401
