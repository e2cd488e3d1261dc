"""MI355X (gfx950) implementation of the PDNQP hot path: the restarted
accelerated PDHG inner solve of the residual-form proximal augmented-
Lagrangian QP subproblem, with the outer multiplier and penalty updates
that drive it.  The compute lives in ``libpdnqp.so`` (HIP); ``pdnqp`` is
its Python binding."""

from .pdnqp import (Solver, default_settings, load, solve_batch, PdnqpError,  # noqa: F401
                    batch_report, batch_set_config, batch_autotune, BATCH_CONFIGS,
                    mlp_forward, mlp_gradient, mlp_gradient_noalloc, mlp_train, MLP_PARAMS,
                    probe_gather,
                    SOLVED, MAX_ITER, TIME_LIMIT, NUMERICAL_ERROR, INACCURATE, STATUS_NAMES,
                    SCALE_RUIZ_A, SCALE_NONE, SCALE_RUIZ_QA, FP64, FP32)
