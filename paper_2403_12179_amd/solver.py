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


def _result(info):
    return SolveResult(info.status, info.cycles, info.levels, info.rel_resid_inf, info.resid_l2, info.f_inf,
                       info.seconds, list(info.hist[:info.nhist]), list(info.hist_l2[:info.nhist]))


def mlmg_solve(phi: MultiFab, rhs: MultiFab, beta: MultiFab | None = None, raise_on_error=True, **params):
    """Solve div(beta grad phi) = rhs (beta=None: Poisson) in place on phi.

    params: nu1, nu2, max_cycles, precision (0 FP64, 1 FP32 V-cycle inside
    FP64 refinement), prolong (2 trilinear, 1 constant), fixed_cycles,
    rel_tol, abs_tol, dx, bottom_rtol, krylov (1: conjugate gradients
    preconditioned by one V-cycle per iteration)."""
    p = solve_params(**params)
    info = L.SolveInfo()
    st = L.lib().bxmg_mlmg_solve(phi.ctx._h, C.byref(p), phi._h, rhs._h, beta._h if beta is not None else None,
                                 C.byref(info))
    res = _result(info)
    if raise_on_error and st not in (0, -4, -5):
        L.check(st)
    return res


def heat_step(u: MultiFab, dt, beta: MultiFab | None = None, source: MultiFab | None = None, raise_on_error=True,
              **params):
    """One backward-Euler step of u_t = div(beta grad u) + source, in place
    on u (a Helmholtz solve with alpha = 1/dt started from u).  params as
    for mlmg_solve (alpha is set by dt)."""
    p = solve_params(**params)
    info = L.SolveInfo()
    st = L.lib().bxmg_heat_step(u.ctx._h, C.byref(p), u._h, source._h if source is not None else None,
                                beta._h if beta is not None else None, float(dt), C.byref(info))
    res = _result(info)
    if raise_on_error and st not in (0, -4, -5):
        L.check(st)
    return res


def heat_run(u: MultiFab, dt, nsteps, beta: MultiFab | None = None, source: MultiFab | None = None, **params):
    """nsteps heat steps on the device-resident u; returns their results."""
    return [heat_step(u, dt, beta, source, **params) for _ in range(int(nsteps))]


def nodal_solve(ba, phi, rhs, raise_on_error=True, **params):
    """Nodal-centred Poisson solve on ba's domain, in place on phi.  phi and
    rhs: contiguous float64 CUDA tensors of shape (n2+1, n1+1, n0+1), i.e.
    indexed [k, j, i] (the F-order node arrays of bxmg_nodal_solve); phi
    holds the initial guess.  params as for mlmg_solve."""
    shape = tuple(ba.domain.size[d] + 1 for d in (2, 1, 0))
    for t in (phi, rhs):
        if tuple(t.shape) != shape or not t.is_contiguous() or t.element_size() != 8 or not t.is_cuda:
            raise ValueError("nodal arrays must be contiguous float64 CUDA tensors of shape %s" % (shape,))
    p = solve_params(**params)
    info = L.SolveInfo()
    ctx = _ctx_of(phi)
    st = L.lib().bxmg_nodal_solve(ctx._h, C.byref(p), ba._h, C.c_void_p(phi.data_ptr()), C.c_void_p(rhs.data_ptr()),
                                  C.byref(info))
    res = _result(info)
    if raise_on_error and st not in (0, -4, -5):
        L.check(st)
    return res


def composite_solve(phi_c: MultiFab, rhs_c: MultiFab, phi_f: MultiFab, rhs_f: MultiFab, raise_on_error=True,
                    **params):
    """Two-level composite Poisson solve (coarse level over the domain, fine
    level of ratio 2 over phi_f's boxes) into phi_c and phi_f, both started
    from zero.  phi_f's BoxArray has the coarse domain refined by 2; its
    boxes are unions of whole coarse cells, 4 fine cells inside the domain.
    params as for mlmg_solve (FP64 V-cycles of the Poisson operator)."""
    p = solve_params(**params)
    info = L.SolveInfo()
    st = L.lib().bxmg_composite_solve(phi_c.ctx._h, C.byref(p), phi_c._h, rhs_c._h, phi_f._h, rhs_f._h,
                                      C.byref(info))
    res = _result(info)
    if raise_on_error and st not in (0, -4, -5):
        L.check(st)
    return res


def _ctx_of(t):
    from .core import default_context
    ctx = default_context()
    if ctx.device != t.device.index:
        raise ValueError("tensor on another device than the default context")
    return ctx


def autotune(phi, rhs, beta=None, cycles=2, **params):
    """Time every candidate launch shape on this problem and keep the fastest
    on phi's context; returns the chosen knobs and the time per V-cycle.
    phi is overwritten."""
    p = solve_params(**params)
    best = (C.c_int32 * 4)()
    ms = C.c_double()
    n = C.c_int32()
    L.check(L.lib().bxmg_autotune(phi.ctx._h, C.byref(p), phi._h, rhs._h, beta._h if beta is not None else None,
                                  int(cycles), best, C.byref(ms), C.byref(n)))
    return {"planes_per_thread": best[0], "buffer_addressing": best[2], "tile_rows_log2_cap": best[3],
            "ms_per_cycle": ms.value, "candidates": n.value}


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


class Batch:
    """Many independent solves in flight together (bxmg_batch_*).

    Batch(ctx, budget_bytes, max_problems, var=False, **params); add() admits a
    problem (None when it does not fit now), step() runs cycles and returns
    the number still running, poll() returns finished (id, SolveResult)."""

    def __init__(self, ctx, budget_bytes, max_problems, var=False, graph=True, **params):
        self.ctx = ctx
        p = solve_params(**params)
        h = C.c_void_p()
        L.check(L.lib().bxmg_batch_create(ctx._h, int(budget_bytes), int(max_problems), 1 if var else 0,
                                          C.byref(p), C.byref(h)))
        self._h = h
        if not graph:
            self.set_graph(False)

    def close(self):
        if self._h:
            L.lib().bxmg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, on):
        L.check(L.lib().bxmg_batch_set(self._h, 0, 1 if on else 0))

    def footprint(self, ba):
        return int(L.lib().bxmg_batch_footprint(self._h, ba._h))

    def add(self, phi, rhs, beta=None, rel_tol=0.0):
        """Problem id, or None if it does not fit now (EBUSY)."""
        pid = C.c_int64()
        st = L.lib().bxmg_batch_add(self._h, phi._h, rhs._h, beta._h if beta is not None else None, float(rel_tol),
                                    C.byref(pid))
        if st == -6:
            return None
        L.check(st)
        return pid.value

    def step(self, ncycles=1):
        n = C.c_int32()
        L.check(L.lib().bxmg_batch_step(self._h, int(ncycles), C.byref(n)))
        return n.value

    def launch(self, ncycles=1):
        """Enqueue ncycles cycles without waiting (pair with collect())."""
        L.check(L.lib().bxmg_batch_launch(self._h, int(ncycles)))

    def collect(self):
        """Wait for the launched cycles; returns the number still running."""
        n = C.c_int32()
        L.check(L.lib().bxmg_batch_collect(self._h, C.byref(n)))
        return n.value

    def poll(self, max_results=None):
        """Finished problems [(id, SolveResult)], oldest first (all of them
        when max_results is None), in chunks of at most 64 per library call."""
        out = []
        chunk = 64
        ids = (C.c_int64 * chunk)()
        infos = (L.SolveInfo * chunk)()
        while max_results is None or len(out) < max_results:
            want = chunk if max_results is None else min(chunk, max_results - len(out))
            n = C.c_int32()
            L.check(L.lib().bxmg_batch_poll(self._h, int(want), ids, infos, C.byref(n)))
            out += [(ids[i], _result(infos[i])) for i in range(n.value)]
            if n.value < want:
                break
        return out

    def remove(self, pid):
        L.check(L.lib().bxmg_batch_remove(self._h, int(pid)))

    def stats(self):
        used, budget = C.c_size_t(), C.c_size_t()
        run, q = C.c_int32(), C.c_int32()
        L.check(L.lib().bxmg_batch_stats(self._h, C.byref(used), C.byref(budget), C.byref(run), C.byref(q)))
        return {"bytes_used": used.value, "bytes_budget": budget.value, "running": run.value, "queued": q.value}

    def run(self, chunk=2):
        """Steps until nothing runs; returns every finished (id, SolveResult)."""
        out = []
        while True:
            n = self.step(chunk)
            out += self.poll()
            if n == 0:
                return out
