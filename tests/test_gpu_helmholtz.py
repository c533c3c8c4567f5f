"""GPU parity of the Helmholtz solve (alpha > 0) and of backward-Euler heat
steps against the oracle, through the C ABI.

Bar as for the Poisson solves: the solution meets the tolerance by the
oracle's FP64 operator (with alpha), agrees with the oracle's solution within
the error bound of that residual, cycle counts within 1 (V-cycle) or 2 (CG),
and with the FP64 V-cycle the iterates of fixed cycles agree with the
oracle's to 1e-12 (the stages are bitwise, the bottom CG sums in another
order).  Closed forms: the sine mode's solution -s/(lam+alpha) and its
decay 1/(1+dt lam) per heat step; a periodic constant right-hand side gives
u = -c/alpha (the operator is not singular).
"""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bx():
    import paper_2403_12179_amd as bx
    return bx


def setup(bx, n, per, mb, f=None, beta=None):
    bc = tuple(bx.PERIODIC if p else bx.DIRICHLET0 for p in per)
    ba = bx.BoxArray.chop((0, 0, 0), (n - 1,) * 3, mb, bc=bc)
    phi = bx.MultiFab(ba).set_val(0.0)
    rhs = bx.MultiFab(ba).set_val(0.0)
    if f is not None:
        rhs.from_global(f)
    bmf = bx.MultiFab(ba).set_val(1.0).from_global(beta) if beta is not None else None
    return ba, phi, rhs, bmf


def lam(n, periodic):
    k = 2 * np.pi if periodic else np.pi
    return 12.0 * np.sin(k / n / 2) ** 2 * n * n


CASES = [  # n, periodic, max_box, var, alpha
    (64, (0, 0, 0), 32, True, 50.0),
    (64, (1, 1, 1), 16, False, 1e3),
    (48, (1, 0, 0), 16, True, 5.0),
]


@pytest.mark.parametrize("n,per,mb,var,alpha", CASES)
@pytest.mark.parametrize("precision,krylov", [(0, 0), (1, 0), (1, 1)])
def test_helmholtz_matches_oracle(bx, orc, n, per, mb, var, alpha, precision, krylov):
    f = W.uniform_rhs((n, n, n), 91)
    beta = W.smooth_gaussian_beta((n, n, n), 92) if var else None
    ba, phi, rhs, bmf = setup(bx, n, per, mb, f, beta)
    res = bx.mlmg_solve(phi, rhs, bmf, alpha=alpha, precision=precision, krylov=krylov)
    assert res.ok, res
    u = phi.to_global()
    dlo, dhi = (0, 0, 0), (n - 1,) * 3
    r = f - orc.apply_op(dlo, dhi, per, 1.0 / n, u, beta, alpha)
    assert np.max(np.abs(r)) <= 1e-10 * np.max(np.abs(f))
    boxes = [(b.small, b.big) for b in ba.boxes]
    uo, io = orc.solve(dlo, dhi, per, boxes, f, beta, alpha=alpha, precision=precision, krylov=krylov)
    assert abs(res.cycles - io["cycles"]) <= (2 if krylov else 1), (res.cycles, io["cycles"])
    kappa = 0.405 * n * n * ((beta.max() / beta.min()) if var else 1.0)
    assert np.max(np.abs(u - uo)) <= kappa * 2e-10 * np.max(np.abs(uo))
    if precision == 0 and krylov == 0:
        phi.set_val(0.0)
        bx.mlmg_solve(phi, rhs, bmf, alpha=alpha, fixed_cycles=3)
        u3, _ = orc.solve(dlo, dhi, per, boxes, f, beta, alpha=alpha, fixed_cycles=3)
        assert np.max(np.abs(phi.to_global() - u3)) <= 1e-12 * np.max(np.abs(u3))


@pytest.mark.parametrize("periodic", [True, False])
def test_helmholtz_sine_closed_form(bx, periodic):
    n = 32
    _, s = W.sine_rhs(n, periodic)
    per = (1, 1, 1) if periodic else (0, 0, 0)
    ba, phi, rhs, _ = setup(bx, n, per, 16, s)
    for alpha in (10.0, 1e4):
        phi.set_val(0.0)
        res = bx.mlmg_solve(phi, rhs, alpha=alpha)
        assert res.ok
        ue = -s / (lam(n, periodic) + alpha)
        assert np.max(np.abs(phi.to_global() - ue)) <= 1e-9 * np.max(np.abs(ue))


def test_periodic_constant_rhs(bx):
    n = 32
    ba, phi, rhs, _ = setup(bx, n, (1, 1, 1), 16)
    rhs.set_val(2.0)
    res = bx.mlmg_solve(phi, rhs, alpha=4.0)
    assert res.ok
    assert np.max(np.abs(phi.to_global() + 0.5)) <= 1e-10


@pytest.mark.parametrize("periodic", [True, False])
def test_heat_steps_decay_the_sine_mode(bx, periodic):
    n = 32
    _, s = W.sine_rhs(n, periodic)
    per = (1, 1, 1) if periodic else (0, 0, 0)
    ba, u, _, _ = setup(bx, n, per, 16)
    u.from_global(s)
    dt = 2e-3
    g = 1.0 / (1.0 + dt * lam(n, periodic))
    for step, res in enumerate(bx.heat_run(u, dt, 3), start=1):
        assert res.ok
    assert np.max(np.abs(u.to_global() - g ** 3 * s)) <= 1e-9 * g ** 3


@pytest.mark.parametrize("precision,krylov", [(0, 0), (1, 1)])
def test_heat_steps_match_oracle(bx, orc, precision, krylov):
    """Three steps with a variable coefficient and a source on a Dirichlet
    48^3 domain in 27 boxes: each GPU state against the oracle's step from
    the same previous state."""
    n = 48
    dlo, dhi = (0, 0, 0), (n - 1,) * 3
    beta = W.smooth_gaussian_beta((n, n, n), 93)
    src = W.uniform_rhs((n, n, n), 94)
    _, s = W.sine_rhs(n, False)
    ba, u, _, bmf = setup(bx, n, (0, 0, 0), 16, None, beta)
    smf = bx.MultiFab(ba, nghost=0).from_global(src)
    u.from_global(s)
    boxes = [(b.small, b.big) for b in ba.boxes]
    dt = 1e-3
    prev = s
    for _ in range(3):
        res = bx.heat_step(u, dt, bmf, smf, precision=precision, krylov=krylov)
        assert res.ok, res
        ug = u.to_global()
        uo, io = orc.heat_step(dlo, dhi, (0, 0, 0), boxes, prev, dt, source=src, beta_glob=beta,
                               precision=precision, krylov=krylov)
        f = -(prev * (1.0 / dt) + src)
        r = f - orc.apply_op(dlo, dhi, (0, 0, 0), 1.0 / n, ug, beta, 1.0 / dt)
        assert np.max(np.abs(r)) <= 1e-10 * np.max(np.abs(f))
        assert abs(res.cycles - io["cycles"]) <= (2 if krylov else 1)
        assert np.max(np.abs(ug - uo)) <= 1e-8 * np.max(np.abs(uo))
        prev = ug


def test_heat_and_alpha_arguments(bx):
    n = 16
    ba, u, rhs, _ = setup(bx, n, (0, 0, 0), 8)
    lib = bx.lib()
    info = bx._lib.SolveInfo()
    p = bx.solve_params()
    for dt in (0.0, -1.0, float("inf")):
        assert lib.bxmg_heat_step(u.ctx._h, C.byref(p), u._h, None, None, dt, C.byref(info)) == -1
    p = bx.solve_params(alpha=-1.0)
    assert lib.bxmg_mlmg_solve(u.ctx._h, C.byref(p), u._h, rhs._h, None, C.byref(info)) == -1
    # batches solve the Poisson operator only
    p = bx.solve_params(alpha=2.0)
    h = C.c_void_p()
    assert lib.bxmg_batch_create(u.ctx._h, 1 << 26, 4, 0, C.byref(p), C.byref(h)) == -1
    # f = 0 gives u = 0 whatever the guess
    u.set_val(3.0)
    res = bx.mlmg_solve(u, rhs, alpha=1.0)
    assert res.ok and res.cycles == 0 and not np.any(u.to_global())
