"""Oracle pins for the Helmholtz operator div(beta grad u) - alpha u and the
backward-Euler heat step built on it.

* The operator: L_alpha u = L_0 u - alpha u on random fields (sign and scale
  of the new term), and the matrix stays symmetric and negative definite.
* Closed forms: the sine product s is an eigenvector of the discrete
  Laplacian, L_h s = -lam s with lam = 12 sin^2(k h / 2) / h^2, so the
  discrete solution of (L_h - alpha) u = s is u = -s / (lam + alpha), for
  both boundary conditions and any alpha.  With alpha > 0 a fully periodic
  problem is no longer singular: f = c gives u = -c / alpha (no mean removed).
* Dense direct solves on 8^3 with alpha (numpy.linalg.solve).
* Heat steps: one step multiplies the sine mode by 1 / (1 + dt lam) exactly,
  and a source s from zero gives dt s / (1 + dt lam); the step starts from
  the previous state, which saves cycles.
"""
import numpy as np
import pytest

import workloads as W
from test_oracle_operator import assemble


def cube(n):
    return (0, 0, 0), (n - 1, n - 1, n - 1)


def lam(n, periodic):
    k = 2 * np.pi if periodic else np.pi
    return 12.0 * np.sin(k / n / 2) ** 2 * n * n


@pytest.mark.parametrize("periodic,var", [((1, 1, 1), False), ((0, 0, 0), True), ((1, 0, 1), True)])
def test_operator_alpha_term(orc, periodic, var):
    n = 12
    lo, hi = cube(n)
    u = W.uniform_rhs((n, n, n), 3)
    beta = W.smooth_gaussian_beta((n, n, n), 4) if var else None
    for alpha in (0.5, 7.0, 3e3):
        a = orc.apply_op(lo, hi, periodic, 1.0 / n, u, beta, alpha)
        b = orc.apply_op(lo, hi, periodic, 1.0 / n, u, beta) - alpha * u
        scale = (12.0 * n * n * (beta.max() if var else 1.0) + alpha) * np.abs(u).max()
        assert np.max(np.abs(a - b)) <= 1e-14 * scale
    A = assemble(orc, (6, 6, 6), periodic, 1.0 / 6, None, 2.5)
    assert np.allclose(A, A.T, atol=0, rtol=1e-14)
    assert np.linalg.eigvalsh(A).max() < 0.0  # definite even when fully periodic


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("alpha", [0.0, 10.0, 1e4])
def test_sine_closed_form(orc, periodic, alpha):
    n = 32
    lo, hi = cube(n)
    _, s = W.sine_rhs(n, periodic)
    per = (1, 1, 1) if periodic else (0, 0, 0)
    u, info = orc.solve(lo, hi, per, orc.chop(lo, hi, 16), s, alpha=alpha)
    assert info["status"] == 0
    ue = -s / (lam(n, periodic) + alpha)
    assert np.max(np.abs(u - ue)) <= 1e-9 * np.max(np.abs(ue))


def test_periodic_constant_solution(orc):
    n = 16
    lo, hi = cube(n)
    u, info = orc.solve(lo, hi, (1, 1, 1), orc.chop(lo, hi, 8), np.full((n, n, n), 2.0, order="F"), alpha=4.0)
    assert info["status"] == 0
    assert np.max(np.abs(u + 0.5)) <= 1e-10


@pytest.mark.parametrize("case,alpha", [("dir_var", 5.0), ("per_const", 20.0), ("mixed_var", 0.5), ("per_var", 1e3)])
def test_dense_direct_8cubed(orc, case, alpha):
    n = 8
    lo, hi = cube(n)
    shape = (n, n, n)
    per = {"dir_var": (0, 0, 0), "per_const": (1, 1, 1), "mixed_var": (1, 0, 0), "per_var": (1, 1, 1)}[case]
    beta = W.smooth_gaussian_beta(shape, 31) if "var" in case else None
    f = W.uniform_rhs(shape, 30)
    for krylov in (0, 1):
        u, info = orc.solve(lo, hi, per, orc.chop(lo, hi, 4), f, beta, rel_tol=1e-12, alpha=alpha, krylov=krylov)
        assert info["status"] == 0
        A = assemble(orc, shape, per, 1.0 / n, beta, alpha)
        ud = np.linalg.solve(A, f.ravel(order="F")).reshape(shape, order="F")
        assert np.max(np.abs(u - ud)) <= 1e-9 * np.max(np.abs(ud))


@pytest.mark.parametrize("periodic", [True, False])
def test_heat_step_decays_the_sine_mode(orc, periodic):
    n = 32
    lo, hi = cube(n)
    per = (1, 1, 1) if periodic else (0, 0, 0)
    boxes = orc.chop(lo, hi, 16)
    _, s = W.sine_rhs(n, periodic)
    dt = 2e-3
    g = 1.0 / (1.0 + dt * lam(n, periodic))
    u = s.copy()
    for step in range(1, 4):
        u, info = orc.heat_step(lo, hi, per, boxes, u, dt)
        assert info["status"] == 0
        assert np.max(np.abs(u - g ** step * s)) <= 1e-9 * g ** step
    # a source from zero: dt s / (1 + dt lam)
    u, info = orc.heat_step(lo, hi, per, boxes, np.zeros((n, n, n), order="F"), dt, source=s)
    assert np.max(np.abs(u - dt * g * s)) <= 1e-9 * dt * g


def test_heat_step_starts_from_the_state(orc):
    n = 32
    lo, hi = cube(n)
    boxes = orc.chop(lo, hi, 16)
    beta = W.smooth_gaussian_beta((n, n, n), 7)
    _, s = W.sine_rhs(n, False)
    u0 = s + 0.01 * W.smooth_gaussian_beta((n, n, n), 8)  # a smooth state (measured: 11 against 13 cycles)
    dt = 1e-3
    u1, i1 = orc.heat_step(lo, hi, (0, 0, 0), boxes, u0, dt, beta_glob=beta)
    # the same Helmholtz solve from zero reaches the same state, in more cycles
    f = -(u0 * (1.0 / dt))
    u1z, iz = orc.solve(lo, hi, (0, 0, 0), boxes, f, beta, alpha=1.0 / dt)
    assert i1["status"] == 0 and iz["status"] == 0 and i1["cycles"] < iz["cycles"]
    assert np.max(np.abs(u1 - u1z)) <= 1e-8 * np.max(np.abs(u1z))
    r = f - orc.apply_op(lo, hi, (0, 0, 0), 1.0 / n, u1, beta, 1.0 / dt)
    assert np.max(np.abs(r)) <= 1e-10 * np.max(np.abs(f))
