"""Oracle pins for the multigrid-preconditioned conjugate gradient solver
(krylov=1: flexible CG, one V-cycle from zero as the preconditioner per
iteration).

* Dense direct solves on 8^3: the PCG solution (FP64 or FP32 V-cycle as the
  preconditioner) equals numpy.linalg.solve / lstsq on the operator matrix.
* Exact preconditioner: on a domain that is its own bottom level the V-cycle
  is the CG bottom solve, i.e. the inverse of the operator to rounding; the
  first iteration must then land on the solution (alpha = 1), so one
  iteration meets a tolerance near machine precision.
* Acceleration: on a rough lognormal coefficient, where the stationary
  V-cycle iteration contracts slowly, the Krylov iteration needs far fewer
  iterations (frozen from a measurement: 11 against 19 at 32^3); steepest
  descent with the same preconditioner or a wrong-signed beta would not.
* Line search and conjugacy: each step is an exact line search and
  consecutive search directions are conjugate with respect to the assembled
  operator matrix -- the two properties the step length and the flexible
  beta are defined by (checked on the iterates, with the dense matrix).
* The final residual, recomputed with the oracle's operator, meets the
  tolerance; status codes as for the stationary solve.
"""
import numpy as np
import pytest

import workloads as W
from test_oracle_operator import assemble


def cube(n):
    return (0, 0, 0), (n - 1, n - 1, n - 1)


@pytest.mark.parametrize("case", ["dir_const", "dir_var", "per_const", "mixed_var"])
@pytest.mark.parametrize("precision", [0, 1])
def test_pcg_dense_direct_8cubed(orc, case, precision):
    n = 8
    lo, hi = cube(n)
    shape = (n, n, n)
    per = {"dir_const": (0, 0, 0), "dir_var": (0, 0, 0), "per_const": (1, 1, 1), "mixed_var": (1, 0, 0)}[case]
    beta = W.smooth_gaussian_beta(shape, 31) if "var" in case else None
    f = W.uniform_rhs(shape, 30, mean_zero=(per == (1, 1, 1)))
    u, info = orc.solve(lo, hi, per, orc.chop(lo, hi, 4), f, beta, rel_tol=1e-12, krylov=1, precision=precision)
    assert info["status"] == 0
    A = assemble(orc, shape, per, 1.0 / n, beta)
    fv = f.ravel(order="F")
    ud = np.linalg.lstsq(A, fv, rcond=None)[0] if per == (1, 1, 1) else np.linalg.solve(A, fv)
    ud = ud.reshape(shape, order="F")
    assert np.max(np.abs(u - ud)) <= 1e-9 * np.max(np.abs(ud))


@pytest.mark.parametrize("shape,per", [((2, 2, 2), (0, 0, 0)), ((3, 5, 7), (0, 0, 0)), ((3, 5, 7), (1, 1, 1)),
                                       ((5, 5, 5), (1, 0, 1))])
@pytest.mark.parametrize("var", [False, True])
def test_pcg_exact_preconditioner_one_iteration(orc, shape, per, var):
    lo, hi = (0, 0, 0), tuple(x - 1 for x in shape)
    f = W.uniform_rhs(shape, 8, mean_zero=(per == (1, 1, 1)))
    beta = W.smooth_gaussian_beta(shape, 9, passes=0) if var else None
    assert len(orc.hierarchy(lo, hi, [(lo, hi)])) == 1  # the domain is its own bottom
    u, info = orc.solve(lo, hi, per, [(lo, hi)], f, beta, h=0.5, rel_tol=1e-13, bottom_rtol=1e-15, krylov=1)
    assert info["status"] == 0 and info["cycles"] == 1
    A = assemble(orc, shape, per, 0.5, beta)
    fv = f.ravel(order="F")
    ud = np.linalg.lstsq(A, fv, rcond=None)[0] if per == (1, 1, 1) else np.linalg.solve(A, fv)
    assert np.max(np.abs(u.ravel(order="F") - ud)) <= 1e-12 * np.max(np.abs(ud))


@pytest.mark.parametrize("var", [False, True])
def test_pcg_accelerates_the_vcycle_iteration(orc, var):
    n = 32
    lo, hi = cube(n)
    f = W.uniform_rhs((n, n, n), 5)
    beta = W.smooth_gaussian_beta((n, n, n), 6) if var else None
    boxes = orc.chop(lo, hi, 16)
    _, mg = orc.solve(lo, hi, (0, 0, 0), boxes, f, beta)
    u, kr = orc.solve(lo, hi, (0, 0, 0), boxes, f, beta, krylov=1)
    assert mg["status"] == 0 and kr["status"] == 0
    if var:  # measured 11 against 19
        assert kr["cycles"] <= 0.65 * mg["cycles"], (kr["cycles"], mg["cycles"])
    else:  # measured 8 against 10
        assert kr["cycles"] < mg["cycles"]
    r = f - orc.apply_op(lo, hi, (0, 0, 0), 1.0 / n, u, beta)
    assert np.max(np.abs(r)) <= 1e-10 * np.max(np.abs(f))
    assert kr["rel_inf"] == np.max(np.abs(r)) / np.max(np.abs(f))  # the reported residual is f - L u


@pytest.mark.parametrize("periodic", [False, True])
def test_pcg_fp32_preconditioner_reaches_fp64_tolerance(orc, periodic):
    n = 32
    lo, hi = cube(n)
    per = (1, 1, 1) if periodic else (0, 0, 0)
    f = W.uniform_rhs((n, n, n), 12, mean_zero=periodic)
    beta = None if periodic else W.smooth_gaussian_beta((n, n, n), 13)
    boxes = orc.chop(lo, hi, 32)
    u64, i64 = orc.solve(lo, hi, per, boxes, f, beta, krylov=1)
    u32, i32 = orc.solve(lo, hi, per, boxes, f, beta, krylov=1, precision=1)
    assert i32["status"] == 0 and abs(i32["cycles"] - i64["cycles"]) <= 2
    r = f - orc.apply_op(lo, hi, per, 1.0 / n, u32, beta)
    assert np.max(np.abs(r)) <= 1e-10 * np.max(np.abs(f))
    kappa = 0.405 * n * n * ((beta.max() / beta.min()) if beta is not None else 1.0)
    assert np.max(np.abs(u32 - u64)) <= kappa * 2e-10 * np.max(np.abs(u64))
    if periodic:
        assert abs(u32.mean()) <= 1e-14 * np.max(np.abs(u32))


def test_pcg_status_codes(orc):
    n = 16
    lo, hi = cube(n)
    boxes = orc.chop(lo, hi, 16)
    f = W.uniform_rhs((n, n, n), 1)
    bad = f.copy()
    bad[3, 4, 5] = np.nan
    _, info = orc.solve(lo, hi, (0, 0, 0), boxes, bad, krylov=1)
    assert info["status"] == -5
    _, info = orc.solve(lo, hi, (0, 0, 0), boxes, f, max_cycles=1, rel_tol=1e-14, krylov=1)
    assert info["status"] == -4 and info["cycles"] == 1
    _, info = orc.solve(lo, hi, (0, 0, 0), boxes, f, fixed_cycles=3, krylov=1)
    assert info["status"] == 0 and info["cycles"] == 3 and len(info["hist"]) == 4
    u, info = orc.solve(lo, hi, (0, 0, 0), boxes, np.zeros((n, n, n), order="F"), krylov=1)
    assert info["status"] == 0 and info["cycles"] == 0 and not u.any()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("per,var", [((0, 0, 0), True), ((1, 1, 1), False)])
def test_pcg_exact_line_search_and_conjugate_directions(orc, precision, per, var):
    """The two properties that define the iteration, checked on its iterates
    with the assembled operator matrix L: each step u_{k+1} - u_k = alpha p_k
    is an exact line search (the new residual f - L u_{k+1} is orthogonal to
    it) and consecutive directions are L-conjugate (p_{k+1} . L p_k = 0, the
    flexible beta).  Iterates come from separate runs of k fixed iterations."""
    n = 8
    lo, hi = cube(n)
    shape = (n, n, n)
    beta = W.smooth_gaussian_beta(shape, 17) if var else None
    f = W.uniform_rhs(shape, 16, mean_zero=(per == (1, 1, 1)))
    A = assemble(orc, shape, per, 1.0 / n, beta)
    boxes = orc.chop(lo, hi, 4)
    us = [np.zeros(n ** 3)]
    for k in range(1, 6):
        u, info = orc.solve(lo, hi, per, boxes, f, beta, fixed_cycles=k, krylov=1, precision=precision)
        assert info["cycles"] == k
        # periodic: each run reports its mean-zero representative; the
        # constants it shifts by are in the null space of the symmetric L
        us.append(u.ravel(order="F"))
    fv = f.ravel(order="F")
    d = [us[k + 1] - us[k] for k in range(5)]
    for k in range(4):
        r1 = fv - A @ us[k + 1]
        ls = abs(r1 @ d[k]) / (np.linalg.norm(r1) * np.linalg.norm(d[k]))
        Ad = A @ d[k]
        cj = abs(d[k + 1] @ Ad) / (np.linalg.norm(d[k + 1]) * np.linalg.norm(Ad))
        assert ls <= 1e-9, (k, ls)
        assert cj <= 1e-9, (k, cj)
