"""Strang splitting on rank-1 / rank-2 lattices for the TDSE on MI355X.

Python face of the HIP library (include/lattice_tdse.h): plans, runs,
adjoints, batched runs, fourth-order compositions, time-dependent
potentials, norm / energy diagnostics and the initial discretization
error, plus a torch.autograd.Function.
All arithmetic of a run happens in the library's HIP kernels.
"""
from ._capi import (LT_C64, LT_C128, LT_KIND_COLUMN, LT_KIND_RESIDENT, LT_KIND_ROW, LatticeError,
                    Plan, lattice_diagnostics, lattice_diagnostics_workspace_size, lattice_plan,
                    lattice_projection_error, lattice_projection_error_workspace_size,
                    lattice_plan_autotune, lattice_plan_get_kernels, lattice_plan_get_kernels_batch,
                    lattice_plan_info, lattice_plan_keys, lattice_plan_points, lattice_plan_set_kernels,
                    lt_timing_enable, lt_timing_summary, num_checkpoints, splitting_run,
                    splitting_times, splitting_workspace_size, strang_adjoint,
                    strang_adjoint_workspace_size, strang_batched_workspace_size, strang_run,
                    strang_run_batched, strang_run_sums, strang_run_sums_workspace_size,
                    strang_workspace_size, Batch, strang_batch_create, strang_batch_run,
                    strang_batch_autotune, strang_batch_kernels, strang_run_noalloc,
                    strang_run_noalloc_capacity)
from .autograd import LatticeStrang, lattice_strang

__all__ = ["LT_C64", "LT_C128", "LatticeError", "Plan", "lattice_plan", "lattice_plan_info",
           "lattice_plan_keys", "lattice_plan_points", "num_checkpoints", "strang_run",
           "strang_adjoint", "strang_run_batched", "strang_workspace_size",
           "strang_adjoint_workspace_size", "strang_batched_workspace_size", "LatticeStrang",
           "lattice_strang", "lt_timing_enable", "lt_timing_summary", "LT_KIND_COLUMN",
           "LT_KIND_ROW", "LT_KIND_RESIDENT", "lattice_plan_autotune", "lattice_plan_set_kernels",
           "lattice_plan_get_kernels", "lattice_plan_get_kernels_batch", "lattice_diagnostics",
           "lattice_diagnostics_workspace_size",
           "splitting_run", "splitting_workspace_size", "splitting_times", "lattice_projection_error",
           "lattice_projection_error_workspace_size", "strang_run_sums", "strang_run_sums_workspace_size",
           "Batch", "strang_batch_create", "strang_batch_run", "strang_batch_autotune", "strang_batch_kernels",
           "strang_run_noalloc", "strang_run_noalloc_capacity"]
