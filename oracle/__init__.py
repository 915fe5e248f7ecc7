"""FP64 CPU oracle for compressed NeNMF -- test infrastructure only.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import this package.  See oracle/nenmf.py for what each function follows.
"""
from .nenmf import (  # noqa: F401
    STOP_GLOBAL, STOP_SUBPROBLEM, OrthBreakdown, RSIResult, NeNMFResult,
    alpha_series, momentum_weights, orth, rsi, lipschitz, gradient,
    projected_gradient, pg_norm, nesterov_nnls, g_data_plain, f_data_plain,
    g_data_compressed, f_data_compressed, nenmf, rre, rre_expanded, rre_history, svd_floor,
    bf16_bits, bf16_value, bf16_round, compress_gaussian, compress_power, hals_update,
    mu_update, subproblem_objective,
)
from . import adjoint  # noqa: F401,E402
