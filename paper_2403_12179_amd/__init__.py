"""bxmg: block-structured geometric multigrid for one MI355X (gfx950).

A cell-centred red-black Gauss-Seidel V-cycle over a BoxArray/MultiFab of
many boxes with ghost cells (the data model of arxiv 2403.12179, Section 2),
every stage a hand-written HIP kernel behind the C ABI in include/bxmg.h.
This package is the thin Python layer: argument marshalling, with PyTorch
supplying device memory and streams.  It has no CPU fallback: without the
built library, importing the solver raises.
"""
from ._lib import BxmgError, DIRICHLET0, PERIODIC, lib  # noqa: F401
from .core import Box, BoxArray, Context, MultiFab, default_context  # noqa: F401
from .solver import (Batch, SolveResult, autotune, bottom_solve, composite_solve, gs_colour, heat_run, heat_step,  # noqa: F401
                     mlmg_solve, nodal_solve, prolong_add, residual, restrict, solve_params)
from .serve import Server  # noqa: F401

__version__ = "0.1.0"
