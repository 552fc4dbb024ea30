"""CPU FP64 oracle for the TSM disconnected-loop path (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this package.  The product library never does.
"""

from .oracle import (  # noqa: F401
    build_oracle,
    load_oracle,
    gamma,
    gamma_mu,
    splitmix64_sequence,
    noise_hash,
    noise_codes,
    noise_z4,
    apply_op,
    cgnr,
    loops,
    loops_est,
    loops_deriv,
    tsm,
    set_threads,
    get_threads,
    OP_M,
    OP_MDAG,
    OP_MDAGM,
    OP_HOP,
    STOP_NORMAL,
    STOP_TRUE,
    LOOP_STD,
    LOOP_ONEEND_VV,
    LOOP_ONEEND_GEN,
    LOOP_DERIV,
    layer_weight_count,
    net_weight_count,
    pt_layer,
    pt_net,
    pt_loss_grad,
    fcg,
    fgmres,
)
