"""Multigrid solve and single-level stages (thin wrappers over the C ABI)."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

from . import _lib as L
from .core import MultiFab


@dataclass
class SolveResult:
    status: int
    cycles: int
    levels: int
    rel_resid_inf: float
    resid_l2: float
    f_inf: float
    seconds: float
    hist: list = field(default_factory=list)
    hist_l2: list = field(default_factory=list)

    @property
    def ok(self):
        return self.status == 0


def solve_params(**kw):
    p = L.SolveParams()
    L.lib().bxmg_solve_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError("unknown solve parameter %r" % k)
        setattr(p, k, v)
    return p


def mlmg_solve(phi: MultiFab, rhs: MultiFab, beta: MultiFab | None = None, raise_on_error=True, **params):
    """Solve div(beta grad phi) = rhs (beta=None: Poisson) in place on phi.

    params: nu1, nu2, max_cycles, precision (0 FP64, 1 FP32 V-cycle inside
    FP64 refinement), prolong (2 trilinear, 1 constant), fixed_cycles,
    rel_tol, abs_tol, dx, bottom_rtol."""
    p = solve_params(**params)
    info = L.SolveInfo()
    st = L.lib().bxmg_mlmg_solve(phi.ctx._h, C.byref(p), phi._h, rhs._h, beta._h if beta is not None else None,
                                 C.byref(info))
    res = SolveResult(info.status, info.cycles, info.levels, info.rel_resid_inf, info.resid_l2, info.f_inf,
                      info.seconds, list(info.hist[:info.nhist]), list(info.hist_l2[:info.nhist]))
    if raise_on_error and st not in (0, -4, -5):
        L.check(st)
    return res


def gs_colour(phi, rhs, h, colour, beta=None):
    L.check(L.lib().bxmg_gs_colour(phi.ctx._h, phi._h, rhs._h, beta._h if beta is not None else None, float(h),
                                   int(colour)))


def residual(phi, rhs, h, r, beta=None):
    norms = (C.c_double * 2)()
    L.check(L.lib().bxmg_residual(phi.ctx._h, phi._h, rhs._h, beta._h if beta is not None else None, float(h), r._h,
                                  norms))
    return norms[0], norms[1]


def restrict(fine, coarse):
    L.check(L.lib().bxmg_restrict(fine.ctx._h, fine._h, coarse._h))


def prolong_add(coarse, fine, order=2):
    L.check(L.lib().bxmg_prolong_add(fine.ctx._h, coarse._h, fine._h, int(order)))


def bottom_solve(phi, rhs, h, rtol=1e-12):
    it = C.c_int32()
    L.check(L.lib().bxmg_bottom_solve(phi.ctx._h, phi._h, rhs._h, None, float(h), float(rtol), C.byref(it)))
    return it.value
