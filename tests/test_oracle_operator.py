"""Oracle pins: the 7-point operator, its variable-coefficient form, the
Gauss-Seidel update and the residual.

* Closed form: on the unit cube with h = 1/n, the sine product at cell
  centres is an exact eigenvector of the discrete Laplacian -- periodic
  sin(2 pi x)...: eigenvalue -12 sin^2(pi h)/h^2; homogeneous Dirichlet with
  odd-reflection ghosts, sin(pi x)...: eigenvalue -12 sin^2(pi h/2)/h^2.
* Symmetry of the assembled variable-coefficient matrix and the telescoping
  of the fluxes (periodic: sum of L u is zero), which fail for any face
  indexing mistake.
* beta == 1 reduces the variable-coefficient operator to the constant one
  (harmonic mean of 1 and 1 is 1, the sum of six ones is 6): bitwise.
* A Gauss-Seidel colour update zeroes the residual of that colour up to
  rounding (the update solves each cell's equation with its neighbours fixed).
"""
import numpy as np
import pytest

import workloads as W


def test_periodic_sine_is_eigenvector(orc):
    for n in (8, 16, 32):
        f, s = W.sine_rhs(n, periodic=True)
        h = 1.0 / n
        lam = -12.0 * np.sin(np.pi * h) ** 2 / h ** 2
        Ls = orc.apply_op((0, 0, 0), (n - 1,) * 3, (1, 1, 1), h, s)
        assert np.max(np.abs(Ls - lam * s)) <= 1e-11 * abs(lam)


def test_dirichlet_sine_is_eigenvector(orc):
    for n in (8, 16, 32):
        f, s = W.sine_rhs(n, periodic=False)
        h = 1.0 / n
        lam = -12.0 * np.sin(np.pi * h / 2) ** 2 / h ** 2
        Ls = orc.apply_op((0, 0, 0), (n - 1,) * 3, (0, 0, 0), h, s)
        assert np.max(np.abs(Ls - lam * s)) <= 1e-11 * abs(lam)


def test_mixed_bc_eigenvector(orc):
    # periodic in x (sin 2 pi x), Dirichlet in y, z (sin pi y, sin pi z)
    n = 16
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    s = np.sin(2 * np.pi * x)[:, None, None] * np.sin(np.pi * x)[None, :, None] * np.sin(np.pi * x)[None, None, :]
    s = np.asfortranarray(s)
    lam = -(4 * np.sin(np.pi * h) ** 2 + 8 * np.sin(np.pi * h / 2) ** 2) / h ** 2
    Ls = orc.apply_op((0, 0, 0), (n - 1,) * 3, (1, 0, 0), h, s)
    assert np.max(np.abs(Ls - lam * s)) <= 1e-11 * abs(lam)


def assemble(orc, shape, periodic, h, beta=None):
    N = int(np.prod(shape))
    A = np.zeros((N, N))
    e = np.zeros(shape, order="F")
    for q in range(N):
        e.ravel(order="F")[:] = 0.0
        e.ravel(order="F")[q] = 1.0
        e2 = np.zeros(shape, order="F")
        e2.ravel(order="F")[q] = 1.0
        A[:, q] = orc.apply_op((0, 0, 0), tuple(x - 1 for x in shape), periodic, h, e2, beta).ravel(order="F")
    return A


@pytest.mark.parametrize("periodic", [(0, 0, 0), (1, 1, 1), (1, 0, 1)])
def test_varcoef_matrix_symmetric_and_sign_definite(orc, periodic):
    shape = (4, 6, 5) if periodic == (0, 0, 0) else (4, 6, 4)
    beta = W.smooth_gaussian_beta(shape, 21)
    A = assemble(orc, shape, periodic, 0.25, beta)
    assert np.array_equal(A, A.T)
    ev = np.linalg.eigvalsh(A)
    assert ev.max() <= 1e-9 * abs(ev.min())  # negative (semi)definite
    if periodic == (1, 1, 1):
        assert np.max(np.abs(A.sum(axis=0))) <= 1e-12 * np.abs(A).max()  # constants in the null space


def test_varcoef_flux_telescopes_periodic(orc):
    shape = (8, 8, 8)
    beta = W.smooth_gaussian_beta(shape, 5)
    u = W.uniform_rhs(shape, 6)
    Lu = orc.apply_op((0, 0, 0), (7, 7, 7), (1, 1, 1), 1.0 / 8, u, beta)
    assert abs(Lu.sum()) <= 1e-12 * np.abs(Lu).sum()


def test_varcoef_beta_one_equals_constant(orc):
    shape = (8, 8, 8)
    u = W.uniform_rhs(shape, 7)
    f = W.uniform_rhs(shape, 8)
    for per in [(1, 1, 1), (0, 0, 0)]:
        a = orc.apply_op((0, 0, 0), (7, 7, 7), per, 1.0 / 8, u)
        b = orc.apply_op((0, 0, 0), (7, 7, 7), per, 1.0 / 8, u, np.ones(shape))
        assert np.array_equal(a, b)
        boxes = orc.chop((0, 0, 0), (7, 7, 7), 4)
        U1 = orc.pack(u, (0, 0, 0), boxes, 1)
        U2 = U1.copy()
        F = orc.pack(f, (0, 0, 0), boxes, 1)
        for c in (0, 1):
            orc.fill_boundary((0, 0, 0), (7, 7, 7), per, boxes, 1, U1)
            orc.apply_bc((0, 0, 0), (7, 7, 7), per, boxes, 1, U1)
            orc.fill_boundary((0, 0, 0), (7, 7, 7), per, boxes, 1, U2)
            orc.apply_bc((0, 0, 0), (7, 7, 7), per, boxes, 1, U2)
            orc.gs((0, 0, 0), (7, 7, 7), per, boxes, 1.0 / 8, c, U1, F)
            orc.gs((0, 0, 0), (7, 7, 7), per, boxes, 1.0 / 8, c, U2, F, np.ones(shape))
        assert np.array_equal(U1, U2)


@pytest.mark.parametrize("var", [False, True])
@pytest.mark.parametrize("periodic", [(1, 1, 1), (0, 0, 0)])
def test_gs_zeroes_residual_of_updated_colour(orc, var, periodic):
    # Ghosts (including the Dirichlet -(mirror) ghosts) are refreshed before
    # each colour and held during it, so the update solves every updated
    # cell's equation with exactly those ghosts: the residual evaluated with
    # the same ghosts vanishes on that colour.  After a refresh it still
    # vanishes away from Dirichlet faces (there the ghost mirrors the cell).
    n = 16
    dlo, dhi = (0, 0, 0), (n - 1,) * 3
    boxes = orc.chop(dlo, dhi, 8)
    shape = (n, n, n)
    beta = W.smooth_gaussian_beta(shape, 3) if var else None
    u = orc.pack(W.uniform_rhs(shape, 1), dlo, boxes, 1)
    f = orc.pack(W.uniform_rhs(shape, 2), dlo, boxes, 1)
    h = 1.0 / n
    par = np.add.outer(np.add.outer(np.arange(n), np.arange(n)), np.arange(n)) % 2
    inner = np.zeros(shape, bool)
    inner[1:-1, 1:-1, 1:-1] = True
    if periodic == (1, 1, 1):
        inner[:] = True
    for colour in (0, 1):
        orc.fill_boundary(dlo, dhi, periodic, boxes, 1, u)
        orc.apply_bc(dlo, dhi, periodic, boxes, 1, u)
        orc.gs(dlo, dhi, periodic, boxes, h, colour, u, f, beta)
        ug = orc.unpack_valid(u, dlo, dhi, boxes, 1)
        scale = 12.0 * np.abs(ug).max() / h ** 2 * (np.abs(beta).max() if var else 1.0)
        r, _, _ = orc.residual(dlo, dhi, periodic, boxes, h, u, f, beta)   # same ghosts as the update
        rg = orc.unpack_valid(r, dlo, dhi, boxes, 1)
        assert np.abs(rg[par == colour]).max() <= 1e-13 * scale
        orc.fill_boundary(dlo, dhi, periodic, boxes, 1, u)
        orc.apply_bc(dlo, dhi, periodic, boxes, 1, u)
        r, _, _ = orc.residual(dlo, dhi, periodic, boxes, h, u, f, beta)
        rg = orc.unpack_valid(r, dlo, dhi, boxes, 1)
        assert np.abs(rg[(par == colour) & inner]).max() <= 1e-13 * scale
        assert np.abs(rg[par != colour]).max() > 1e-6  # the other colour is not solved


def test_residual_norms(orc):
    n = 8
    boxes = orc.chop((0, 0, 0), (7, 7, 7), 4)
    u = orc.pack(W.uniform_rhs((n, n, n), 1), (0, 0, 0), boxes, 1)
    f = orc.pack(W.uniform_rhs((n, n, n), 2), (0, 0, 0), boxes, 1)
    orc.fill_boundary((0, 0, 0), (7, 7, 7), (0, 0, 0), boxes, 1, u)
    orc.apply_bc((0, 0, 0), (7, 7, 7), (0, 0, 0), boxes, 1, u)
    r, rinf, rl2 = orc.residual((0, 0, 0), (7, 7, 7), (0, 0, 0), boxes, 1.0 / n, u, f)
    rg = orc.unpack_valid(r, (0, 0, 0), (7, 7, 7), boxes, 1)
    ug = orc.unpack_valid(u, (0, 0, 0), (7, 7, 7), boxes, 1)
    fg = orc.unpack_valid(f, (0, 0, 0), (7, 7, 7), boxes, 1)
    Lu = orc.apply_op((0, 0, 0), (7, 7, 7), (0, 0, 0), 1.0 / n, ug)
    assert np.array_equal(rg, fg - Lu)
    assert rinf == np.abs(rg).max()
    assert np.isclose(rl2, np.sum(rg ** 2), rtol=1e-14)
