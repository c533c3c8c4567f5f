"""Oracle pins for the nodal Poisson solver (node-centred data, nodes at
x = i h, i = 0..n; Dirichlet boundary nodes held at 0, periodic node n = node
0).

* The operator against an independent construction: the Kronecker sum of
  1-D second-difference matrices over the unknown nodes, entry by entry.
* Closed forms: the sine product at the nodes is an eigenvector,
  L s = -12 sin^2(k h / 2) / h^2 s, so f = s gives u = -s / lam; the
  manufactured f = -3 k^2 s converges at second order (errors from the
  eigenvalue, ratio -> 4).
* Transfers: full weighting equals the transpose of trilinear prolongation
  over 8 (inner products over the unknowns), it keeps constants on periodic
  grids, and trilinear prolongation reproduces linear functions exactly.
* Gauss-Seidel zeroes the residual of the colour it updates; the bottom CG
  and whole solves match numpy's dense solves on 8^3 cells; the V-cycle
  contracts at an h-independent rate.
"""
import numpy as np
import pytest

import workloads as W


def nodes(n):
    return tuple(x + 1 for x in n)


def unknown_mask(n, per):
    m = np.ones(nodes(n), bool)
    for d in range(3):
        sl = [slice(None)] * 3
        if per[d]:
            sl[d] = n[d]
            m[tuple(sl)] = False
        else:
            sl[d] = 0
            m[tuple(sl)] = False
            sl[d] = n[d]
            m[tuple(sl)] = False
    return m


def second_diff(m, periodic):
    T = -2.0 * np.eye(m) + np.eye(m, k=1) + np.eye(m, k=-1)
    if periodic:
        T[0, -1] = T[-1, 0] = 1.0
    return T


def kron_matrix(n, per, h):
    """(T_x (+) T_y (+) T_z) / h^2 over the unknowns, x fastest."""
    ms = [n[d] if per[d] else n[d] - 1 for d in range(3)]
    Ts = [second_diff(ms[d], per[d]) for d in range(3)]
    I = [np.eye(m) for m in ms]
    A = np.kron(I[2], np.kron(I[1], Ts[0])) + np.kron(I[2], np.kron(Ts[1], I[0])) + np.kron(Ts[2], np.kron(I[1], I[0]))
    return A / h ** 2


def oracle_matrix(orc, n, per, h):
    mask = unknown_mask(n, per)
    idx = np.flatnonzero(mask.ravel(order="F"))
    A = np.zeros((len(idx), len(idx)))
    for c, q in enumerate(idx):
        e = np.zeros(nodes(n), order="F")
        e.ravel(order="F")[q] = 1.0
        if any(per):  # the periodic copies mirror their node
            e = mirror_copies(e, n, per)
        A[:, c] = orc.nodal_apply(n, per, h, e).ravel(order="F")[idx]
    return A


def mirror_copies(u, n, per):
    u = u.copy(order="F")
    for d in range(3):
        if per[d]:
            src = [slice(None)] * 3
            dst = [slice(None)] * 3
            src[d] = 0
            dst[d] = n[d]
            u[tuple(dst)] = u[tuple(src)]
    return u


def sine(n, per):
    h = 1.0 / n[0]
    out = np.ones(nodes(n))
    ks = []
    for d in range(3):
        k = 2 * np.pi if per[d] else np.pi
        ks.append(k)
        x = np.arange(n[d] + 1) * h
        shape = [1, 1, 1]
        shape[d] = n[d] + 1
        out = out * np.sin(k * x).reshape(shape)
    lam = sum(4.0 * np.sin(k * h / 2) ** 2 / h ** 2 for k in ks)
    return np.asfortranarray(out), lam, ks


@pytest.mark.parametrize("per", [(0, 0, 0), (1, 1, 1), (1, 0, 1)])
def test_operator_is_kronecker_sum(orc, per):
    n = (6, 4, 8) if per != (1, 1, 1) else (4, 6, 4)
    h = 0.25
    A = oracle_matrix(orc, n, per, h)
    assert np.array_equal(A, kron_matrix(n, per, h))


@pytest.mark.parametrize("per", [(0, 0, 0), (1, 1, 1), (0, 1, 0)])
@pytest.mark.parametrize("m", [16, 32])
def test_sine_closed_form(orc, per, m):
    n = (m, m, m)
    s, lam, _ = sine(n, per)
    u, info = orc.nodal_solve(n, per, s)
    assert info["status"] == 0
    assert np.max(np.abs(u + s / lam)) <= 1e-9 * np.max(np.abs(s)) / lam


@pytest.mark.parametrize("per", [(0, 0, 0), (1, 1, 1)])
def test_second_order_convergence(orc, per):
    errs = []
    for m in (16, 32, 64):
        n = (m, m, m)
        s, lam, ks = sine(n, per)
        k2 = sum(k * k for k in ks)
        u, info = orc.nodal_solve(n, per, -k2 * s)
        e = np.max(np.abs(u - s))
        assert abs(e - abs(k2 / lam - 1.0) * np.max(np.abs(s))) <= 1e-6 * e
        errs.append(e)
    assert 3.9 < errs[0] / errs[1] < 4.1 and 3.95 < errs[1] / errs[2] < 4.05


@pytest.mark.parametrize("per", [(0, 0, 0), (1, 1, 1), (1, 0, 0)])
def test_restriction_is_prolongation_transposed(orc, per):
    n = (8, 12, 8)
    nc = tuple(x // 2 for x in n)
    mf, mc = unknown_mask(n, per), unknown_mask(nc, per)
    rng = np.random.default_rng(5)
    r = np.where(mf, rng.standard_normal(nodes(n)), 0.0)
    e = np.where(mc, rng.standard_normal(nodes(nc)), 0.0)
    r, e = mirror_copies(np.asfortranarray(r), n, per), mirror_copies(np.asfortranarray(e), nc, per)
    Rr = orc.nodal_restrict(n, per, r)
    Pe = orc.nodal_prolong_add(n, per, e, np.zeros(nodes(n), order="F"))
    lhs = np.sum((Rr * e)[mc])
    rhs = np.sum((r * Pe)[mf]) / 8.0
    assert abs(lhs - rhs) <= 1e-13 * np.sum(np.abs(r)) * np.max(np.abs(e))


def test_transfer_exactness(orc):
    n = (8, 8, 8)
    per = (1, 1, 1)
    Rc = orc.nodal_restrict(n, per, np.full(nodes(n), 3.0, order="F"))
    assert np.all(Rc[unknown_mask((4, 4, 4), per)] == 3.0)
    # trilinear prolongation of a linear function (dyadic values) is exact
    nd = (0, 0, 0)
    nc = (4, 4, 4)
    X, Y, Z = np.meshgrid(*[np.arange(x + 1, dtype=float) for x in nc], indexing="ij")
    e = np.asfortranarray(0.5 * X - 0.25 * Y + 2.0 * Z + 1.0)
    Xf, Yf, Zf = np.meshgrid(*[np.arange(x + 1, dtype=float) / 2 for x in n], indexing="ij")
    want = 0.5 * Xf - 0.25 * Yf + 2.0 * Zf + 1.0
    got = orc.nodal_prolong_add(n, nd, e, np.zeros(nodes(n), order="F"))
    m = unknown_mask(n, nd)
    assert np.array_equal(got[m], want[m])


@pytest.mark.parametrize("per", [(0, 0, 0), (1, 1, 1)])
def test_gs_zeroes_residual_of_updated_colour(orc, per):
    n = (16, 16, 16)
    h = 1.0 / 16
    m = unknown_mask(n, per)
    u = mirror_copies(np.asfortranarray(np.where(m, W.uniform_rhs(nodes(n), 1), 0.0)), n, per)
    f = np.asfortranarray(W.uniform_rhs(nodes(n), 2))
    par = np.add.outer(np.add.outer(np.arange(17), np.arange(17)), np.arange(17)) % 2
    for colour in (0, 1):
        u = orc.nodal_gs(n, per, h, colour, u, f)
        r, _, _ = orc.nodal_residual(n, per, h, u, f)
        scale = 12.0 * np.abs(u).max() / h ** 2
        assert np.abs(r[m & (par == colour)]).max() <= 1e-13 * scale
        assert np.abs(r[m & (par != colour)]).max() > 1e-6


@pytest.mark.parametrize("per", [(0, 0, 0), (1, 1, 1), (1, 0, 1)])
def test_dense_direct(orc, per):
    n = (8, 8, 8)
    h = 1.0 / 8
    m = unknown_mask(n, per)
    f = np.asfortranarray(W.uniform_rhs(nodes(n), 9))
    if per == (1, 1, 1):
        f = np.asfortranarray(f - f[m].mean())
    A = kron_matrix(n, per, h)
    fv = f.ravel(order="F")[np.flatnonzero(m.ravel(order="F"))]
    ud = np.linalg.lstsq(A, fv, rcond=None)[0] if per == (1, 1, 1) else np.linalg.solve(A, fv)
    u, info = orc.nodal_solve(n, per, f, rel_tol=1e-12)
    assert info["status"] == 0
    got = u.ravel(order="F")[np.flatnonzero(m.ravel(order="F"))]
    assert np.max(np.abs(got - ud)) <= 1e-9 * np.max(np.abs(ud))
    ub, it = orc.nodal_bottom(n, per, h, f)
    got = ub.ravel(order="F")[np.flatnonzero(m.ravel(order="F"))]
    assert np.max(np.abs(got - ud)) <= 1e-10 * np.max(np.abs(ud)) and it <= 2 * len(fv)


def test_contraction_h_independent(orc):
    worst = []
    for m in (16, 32, 64):
        n = (m, m, m)
        f = np.asfortranarray(W.uniform_rhs(nodes(n), 2))
        _, info = orc.nodal_solve(n, (0, 0, 0), f, fixed_cycles=8)
        h = np.asarray(info["hist"])
        rho = h[1:] / h[:-1]
        assert rho.max() < 0.2
        worst.append(rho[2:].max())
    assert max(worst) / min(worst) <= 1.5


def test_status_codes(orc):
    n = (8, 8, 8)
    f = np.asfortranarray(W.uniform_rhs(nodes(n), 3))
    bad = f.copy()
    bad[3, 3, 3] = np.nan
    assert orc.nodal_solve(n, (0, 0, 0), bad)[1]["status"] == -5
    _, info = orc.nodal_solve(n, (0, 0, 0), f, max_cycles=1, rel_tol=1e-15)
    assert info["status"] == -4 and info["cycles"] == 1
    u, info = orc.nodal_solve(n, (0, 0, 0), np.zeros(nodes(n), order="F"))
    assert info["status"] == 0 and info["cycles"] == 0 and not u.any()
