"""MI355X (gfx950) implementation of the ANOVA-kernel fast summation and
KRR conjugate gradients of Nestler, Stoll and Wagner (arXiv 2111.10140).

The compute path is the HIP library ``libanova.so`` behind the C ABI in
``include/anova.h``; ``_lib`` is its ctypes binding (argument marshalling
only).  ``serve`` holds the request loop that batches CG iterations;
``features`` and ``krr`` the preprocessing and the end-to-end classifier
(fit, predict, grid search) on top of the library.
"""
from . import _lib  # noqa: F401
from ._lib import (ANOVA_FP32_NFFT, ANOVA_FP64, AnovaError, Plan, anova_fastsum_plan,  # noqa: F401
                   anova_last_error, anova_matvec, anova_plan_destroy, anova_stage_convolve,
                   anova_stage_gather, anova_stage_spread, grid_tensor, krr_cg_solve,
                   make_params, anova_predict_plan, anova_predict_plan_host, anova_predict,
                   krr_cg_solve_shifts)
