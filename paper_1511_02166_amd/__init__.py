"""Batched 2-D panel-method solver for AMD MI355X (gfx950).

Thin Python binding over the C ABI of ``libpanel.so`` (declared in
``include/panel.h``).  Every step of the computation runs in the HIP
kernels of that library; this package only marshals arguments (device
pointers of torch tensors, the current HIP stream) and raises on errors.
There is no CPU fallback: if the library is missing, importing the binding
functions raises.
"""
from __future__ import annotations

from ._binding import (  # noqa: F401
    PANEL_FP32_REFINE,
    PANEL_FP64,
    PANEL_HESS_SMITH,
    PANEL_STREAM_FUNCTION,
    PANEL_KMAX,
    PANEL_NMAX,
    PANEL_NMIN,
    PANEL_NOALLOC_MAX_BYTES,
    PANEL_GA_MAX_CTRL,
    PANEL_GA_MAX_DEGREE,
    PANEL_GA_MAX_GENES,
    PANEL_GA_MAX_TOURNAMENT,
    PanelError,
    Plan,
    lib_path,
    load_library,
    panel_adjoint,
    panel_assemble,
    panel_bspline_nodes,
    panel_factor_solve,
    panel_forces,
    panel_ga_fitness,
    panel_ga_init,
    panel_ga_record,
    panel_ga_step,
    panel_ga_uniform_count,
    panel_last_error,
    panel_math_eval,
    panel_naca4,
    panel_naca4_vjp,
    panel_plan_create,
    panel_plan_destroy,
    panel_plan_get_tiling,
    panel_plan_set_formulation,
    panel_plan_set_tiling,
    panel_plan_set_wave_limit,
    panel_solve_noalloc,
    panel_status_str,
    panel_thwaites,
    panel_workspace_init,
    panel_workspace_layout,
    panel_workspace_size,
)
from .solver import PanelSolver, TileTable, naca_cl, panel_cl, panel_cl_cp  # noqa: F401
from .ga import GeneticOptimizer  # noqa: F401

__all__ = [
    "PANEL_FP64", "PANEL_FP32_REFINE", "PANEL_STREAM_FUNCTION", "PANEL_HESS_SMITH", "PANEL_NMAX", "PANEL_NMIN", "PANEL_KMAX",
    "PanelError", "Plan", "PanelSolver", "TileTable", "panel_cl", "panel_cl_cp", "naca_cl",
    "panel_plan_create", "panel_plan_destroy", "panel_plan_set_wave_limit", "panel_plan_set_tiling",
    "panel_plan_get_tiling", "panel_plan_set_formulation", "panel_workspace_size", "panel_workspace_init", "panel_workspace_layout",
    "panel_assemble", "panel_factor_solve", "panel_forces", "panel_adjoint", "panel_naca4",
    "panel_naca4_vjp", "panel_thwaites", "panel_math_eval", "panel_solve_noalloc", "PANEL_NOALLOC_MAX_BYTES", "panel_status_str", "panel_last_error", "load_library", "lib_path",
    "panel_bspline_nodes", "panel_ga_init", "panel_ga_fitness", "panel_ga_uniform_count", "panel_ga_step", "panel_ga_record",
    "PANEL_GA_MAX_GENES", "PANEL_GA_MAX_CTRL", "PANEL_GA_MAX_DEGREE", "PANEL_GA_MAX_TOURNAMENT", "GeneticOptimizer",
]
