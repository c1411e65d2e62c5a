"""SupPCG (superiorized preconditioned conjugate gradients) for least-squares
tomography on AMD Instinct MI355X (gfx950).

The computation lives in ``libsuppcg.so`` (hand-written HIP kernels behind the
C ABI of ``include/suppcg.h``); this package is its PyTorch binding.
"""
from .api import (Context, Geometry, LearnedPrecond, SolveResult, StoredMatrix, SupPCGError, batch_tuning, context,
                  paper_se_axes, sp_backproject, sp_gradient, sp_precond_apply, sp_project, sp_residual,
                  sp_blobart_solve, sp_selective_error, sp_supart_solve, tune_shapes, tuning_clear, tuning_list, tuning_load,
                  tuning_save, tuning_set,
                  sp_solve_status, sp_state_load, sp_state_save, sp_suppcg_solve,
                  sp_suppcg_solve_async, sp_suppcg_solve_batched, sp_tv, sp_tv_grad, sp_tv_perturb)

__all__ = ["Context", "Geometry", "LearnedPrecond", "SolveResult", "StoredMatrix", "SupPCGError", "batch_tuning", "context",
           "paper_se_axes", "sp_suppcg_solve_batched", "sp_backproject", "sp_gradient", "sp_blobart_solve", "sp_selective_error", "sp_supart_solve", "tune_shapes", "tuning_clear", "tuning_list", "tuning_load",
           "tuning_save", "tuning_set",
           "sp_precond_apply", "sp_project", "sp_residual", "sp_solve_status", "sp_state_load",
           "sp_state_save", "sp_suppcg_solve", "sp_suppcg_solve_async", "sp_tv",
           "sp_tv_grad", "sp_tv_perturb"]
