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


def assemble(orc, shape, periodic, h, beta=None, alpha=0.0):
    N = int(np.prod(shape))
    A = np.zeros((N, N))
    e = np.zeros(shape, order="F")
    for q in range(N):
        e.ravel(order="F")[:] = 0.0
        e.ravel(order="F")[q] = 1.0
        e2 = np.zeros(shape, order="F")
        e2.ravel(order="F")[q] = 1.0
        A[:, q] = orc.apply_op((0, 0, 0), tuple(x - 1 for x in shape), periodic, h, e2, beta, alpha).ravel(order="F")
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


@pytest.mark.parametrize("var,alpha", [(False, 0.0), (True, 0.0), (False, 300.0), (True, 5000.0)])
@pytest.mark.parametrize("periodic", [(1, 1, 1), (0, 0, 0)])
def test_gs_zeroes_residual_of_updated_colour(orc, var, periodic, alpha):
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
        orc.gs(dlo, dhi, periodic, boxes, h, colour, u, f, beta, alpha)
        ug = orc.unpack_valid(u, dlo, dhi, boxes, 1)
        scale = (12.0 / h ** 2 + alpha) * np.abs(ug).max() * (np.abs(beta).max() if var else 1.0)
        r, _, _ = orc.residual(dlo, dhi, periodic, boxes, h, u, f, beta, alpha)   # same ghosts as the update
        rg = orc.unpack_valid(r, dlo, dhi, boxes, 1)
        assert np.abs(rg[par == colour]).max() <= 1e-13 * scale
        orc.fill_boundary(dlo, dhi, periodic, boxes, 1, u)
        orc.apply_bc(dlo, dhi, periodic, boxes, 1, u)
        r, _, _ = orc.residual(dlo, dhi, periodic, boxes, h, u, f, beta, alpha)
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


# ------------------------------------------------ variable-coefficient faces
# Independent pins of the face rules (reading R16): a fine face between two
# cells is the conductance of the two half cells in series, 2 / (1/a + 1/b);
# a coarse face is the area mean of the four fine faces it covers.  Both are
# computed here in exact rational arithmetic, not with the oracle's formula.
from fractions import Fraction


def _pow2_beta(shape, seed):
    rng = np.random.default_rng(seed)
    return np.asfortranarray(np.exp2(rng.integers(-4, 5, size=shape)).astype(np.float64))


def _series(a, b):
    return 2 / (1 / Fraction(a) + 1 / Fraction(b))


def _fine_faces_exact(beta, periodic):
    """Level-0 faces from cell beta: series conductance of the two cells; the
    cell beyond a Dirichlet face is the boundary cell itself (no jump across
    the wall), beyond a periodic face the wrapped cell."""
    out = []
    for d in range(3):
        n = beta.shape[d]
        shp = list(beta.shape)
        shp[d] += 1
        F = np.zeros(shp, order="F")
        for idx in np.ndindex(*shp):
            i = idx[d]
            left = list(idx)
            right = list(idx)
            left[d] = i - 1
            if i == 0:
                left[d] = n - 1 if periodic[d] else 0
            if i == n:
                right[d] = 0 if periodic[d] else n - 1
            F[idx] = float(_series(beta[tuple(left)], beta[tuple(right)]))
        out.append(F)
    return out


@pytest.mark.parametrize("periodic", [(0, 0, 0), (1, 0, 1), (1, 1, 1)])
def test_level0_faces_are_series_conductances(orc, periodic):
    # beta = 2^k: 1/a + 1/b is exact, so the oracle's face must be the
    # correctly rounded exact series conductance, bit for bit
    shape = (8, 6, 4)
    beta = _pow2_beta(shape, 5)
    lo, hi = (0, 0, 0), tuple(s - 1 for s in shape)
    got = orc.faces(lo, hi, periodic, [(lo, hi)], beta)[0]
    exp = _fine_faces_exact(beta, periodic)
    for d in range(3):
        assert np.array_equal(got[d], exp[d]), d
    # a wall face carries the boundary cell's own beta
    if not periodic[0]:
        assert np.array_equal(got[0][0], beta[0]) and np.array_equal(got[0][-1], beta[-1])


def test_layered_coefficient_keeps_flux_continuous(orc):
    # beta varies along x only, u is the exact flux-continuous profile of
    # d/dx(beta du/dx) = 0 with unit flux: between two cell centres u rises
    # by h/2 (1/beta_left + 1/beta_right).  The 7-point operator with
    # series-conductance faces maps it to zero at every cell whose x
    # neighbours are both interior (an arithmetic face mean does not).
    n, ny = 16, 4
    h = 1.0 / n
    rng = np.random.default_rng(8)
    b1 = np.exp2(rng.integers(-3, 4, size=n)).astype(np.float64)
    u1 = np.zeros(n)
    for i in range(1, n):
        u1[i] = u1[i - 1] + 0.5 * h * (1.0 / b1[i - 1] + 1.0 / b1[i])
    beta = np.asfortranarray(np.broadcast_to(b1[:, None, None], (n, ny, ny)).copy())
    u = np.asfortranarray(np.broadcast_to(u1[:, None, None], (n, ny, ny)).copy())
    Lu = orc.apply_op((0, 0, 0), (n - 1, ny - 1, ny - 1), (0, 1, 1), h, u, beta)
    assert np.max(np.abs(Lu[1:n - 1])) <= 1e-9 / h
    # and the flux is not zero in the mean: the walls see it
    assert np.min(np.abs(Lu[[0, n - 1]])) > 1.0


@pytest.mark.parametrize("periodic", [(0, 0, 0), (1, 1, 0)])
def test_coarse_faces_are_area_means(orc, periodic):
    # coarse face (d, I) = mean of the 4 fine d-faces at 2I whose tangential
    # indices are (2J, 2J+1) x (2K, 2K+1); checked on levels 1 and 2 against
    # exact rational means of the level above (the oracle rounds the three
    # additions and the scaling: at most a few ulp)
    n = 8
    beta = _pow2_beta((n, n, n), 6)
    lo, hi = (0, 0, 0), (n - 1,) * 3
    levels = orc.faces(lo, hi, periodic, orc.chop(lo, hi, 4), beta)
    assert len(levels) == 3
    for l in (1, 2):
        for d in range(3):
            fine, coarse = levels[l - 1][d], levels[l][d]
            t = [e for e in range(3) if e != d]
            for idx in np.ndindex(*coarse.shape):
                base = [2 * x for x in idx]
                acc = Fraction(0)
                for p in (0, 1):
                    for q in (0, 1):
                        c = list(base)
                        c[t[0]] += p
                        c[t[1]] += q
                        acc += Fraction(fine[tuple(c)])
                exact = acc / 4
                assert abs(Fraction(coarse[idx]) - exact) <= abs(exact) * Fraction(1, 2 ** 50), (l, d, idx)
