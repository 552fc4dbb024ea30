"""MI355X (gfx950) implementation of the truncated-solver-method evaluation
of disconnected quark loops with twisted-mass Wilson fermions
(Alexandrou et al., arXiv:1211.0126).

The computation lives in the HIP library libtmqcd.so (C ABI in
include/tmqcd.h); this package holds its sources (csrc/), the build script
and a thin ctypes binding with the same entry-point names.
"""

from .binding_tuning import tm_set_graphs, tm_profile_entries, tm_set_march, tm_autotune_cg, tm_set_eo_tiles, tm_autotune_eo  # noqa: F401
from .binding import (  # noqa: F401
    Caps,
    Context,
    TmError,
    caps,
    tm_workspace_bytes,
    load_library,
    solve_params,
    tm_abi_version,
    tm_create,
    tm_gauge_load,
    tm_dslash,
    tm_dslash_noalloc,
    tm_field_bytes,
    tm_field_convert,
    tm_noise_z4,
    tsm_solve_batch,
    tsm_contract,
    tsm_loops,
    tm_profile_enable,
    tm_profile_read,
    tm_precond_weight_count,
    tm_precond_set,
    tm_precond_get,
    tm_precond_apply,
    tm_precond_loss_grad,
    tm_precond_train,
    tm_autotune,
    tm_set_lane_rhs,
    SOLVER_CG,
    SOLVER_FCG_LEARNED,
    SOLVER_CG_EO,
    EXPORTS,
    LIB_PATH,
    PREC_F64,
    PREC_F32,
    PREC_F16,
    PREC_BF16,
    OP_M,
    OP_MDAG,
    OP_MDAGM,
    OP_HOP,
    LAYOUT_CANONICAL,
    LAYOUT_NATIVE,
    STOP_NORMAL,
    STOP_TRUE,
    LOOP_STANDARD,
    LOOP_ONEEND_ISOVECTOR,
    LOOP_ONEEND_GENERALIZED,
    LOOP_DERIVATIVE,
)
