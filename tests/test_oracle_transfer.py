"""Oracle pins: restriction (average of the 8 children) and prolongation
(trilinear cell-centred, or piecewise constant).

Independent references: numpy reshape-mean for the restriction; a separable
1D interpolation (weights 3/4 on the parent, 1/4 on the neighbour on the
child's side, applied per direction) on the padded global coarse array for
the prolongation.  Dyadic codes make every result exact, so comparisons are
bitwise whatever the summation order.
"""
import numpy as np
import pytest

import workloads as W
from test_oracle_fill import padded_expect


def restrict_ref(g):
    nx, ny, nz = g.shape
    return g.reshape(nx // 2, 2, ny // 2, 2, nz // 2, 2).mean(axis=(1, 3, 5))


def prolong_ref(c_padded, fine_shape):
    """Separable trilinear interpolation from a coarse array padded by 1."""
    out = c_padded
    for d in range(3):
        n = fine_shape[d]
        i = np.arange(n)
        P = i // 2 + 1  # +1: padding offset
        s = np.where(i % 2 == 1, 1, -1)
        a = np.take(out, P, axis=d)
        b = np.take(out, P + s, axis=d)
        out = 0.75 * a + 0.25 * b
        # keep the padding on the other axes only
    return out


def interior(a):
    return a[1:-1, 1:-1, 1:-1]


@pytest.mark.parametrize("coarse_agglomerated", [False, True])
def test_restriction_vs_reshape_mean(orc, coarse_agglomerated):
    dlo, dhi = (0, 0, 0), (15, 15, 11)
    fb = orc.chop(dlo, dhi, 4)
    cdlo, cdhi = (0, 0, 0), (7, 7, 5)
    cb = [(cdlo, cdhi)] if coarse_agglomerated else [(tuple(x // 2 for x in lo), tuple(x // 2 for x in hi)) for lo, hi in fb]
    g = W.dyadic_codes((16, 16, 12), 4)
    rf = orc.pack(g, dlo, fb, 1)
    fc = orc.restrict(fb, 1, cb, 1, rf)
    got = orc.unpack_valid(fc, cdlo, cdhi, cb, 1)
    assert np.array_equal(got, restrict_ref(g))
    assert np.sum(got) * 8 == np.sum(g)  # mean preserved


def test_restriction_of_constant(orc):
    fb = orc.chop((0, 0, 0), (7, 7, 7), 4)
    cb = [(tuple(x // 2 for x in lo), tuple(x // 2 for x in hi)) for lo, hi in fb]
    g = np.full((8, 8, 8), 0.3, order="F")  # not dyadic: R(c) = c still exact? (8 equal terms, then * 1/8)
    fc = orc.restrict(fb, 1, cb, 1, orc.pack(g, (0, 0, 0), fb, 1))
    got = orc.unpack_valid(fc, (0, 0, 0), (3, 3, 3), cb, 1)
    assert np.all(got == 0.3)


@pytest.mark.parametrize("periodic", [(1, 1, 1), (0, 0, 0), (1, 0, 1)])
@pytest.mark.parametrize("coarse_agglomerated", [False, True])
def test_trilinear_vs_separable(orc, periodic, coarse_agglomerated):
    dlo, dhi = (-8, 0, 0), (7, 11, 15)
    fb = orc.chop(dlo, dhi, 4)
    cdlo, cdhi = (-4, 0, 0), (3, 5, 7)
    cb = [(cdlo, cdhi)] if coarse_agglomerated else [(tuple(x // 2 for x in lo), tuple(x // 2 for x in hi)) for lo, hi in fb]
    cshape = (8, 6, 8)
    c = W.dyadic_codes(cshape, 9)
    ec = orc.pack(c, cdlo, cb, 1)
    orc.fill_boundary(cdlo, cdhi, periodic, cb, 1, ec)
    orc.apply_bc(cdlo, cdhi, periodic, cb, 1, ec)
    base = W.dyadic_codes((16, 12, 16), 10)
    uf = orc.pack(base, dlo, fb, 1)
    orc.prolong(fb, 1, cb, 1, ec, uf, order=2)
    got = orc.unpack_valid(uf, dlo, dhi, fb, 1)
    exp = base + prolong_ref(padded_expect(c, periodic, 1, True), (16, 12, 16))
    assert np.array_equal(got, exp)


def test_trilinear_reproduces_linear(orc):
    # e_c = a + b.x at coarse centres -> fine values a + b.x at fine centres
    n = 16
    h = 1.0 / n
    H = 2 * h
    a, b = 0.5, (1.0, -2.0, 0.25)
    X = [(np.arange(n // 2) + 0.5) * H] * 3
    c = a + b[0] * X[0][:, None, None] + b[1] * X[1][None, :, None] + b[2] * X[2][None, None, :]
    c = np.asfortranarray(c)
    fb = orc.chop((0, 0, 0), (n - 1,) * 3, 8)
    cb = [(tuple(x // 2 for x in lo), tuple(x // 2 for x in hi)) for lo, hi in fb]
    ec = orc.pack(c, (0, 0, 0), cb, 1)
    orc.fill_boundary((0, 0, 0), (n // 2 - 1,) * 3, (0, 0, 0), cb, 1, ec)
    orc.apply_bc((0, 0, 0), (n // 2 - 1,) * 3, (0, 0, 0), cb, 1, ec)
    uf = orc.pack(np.zeros((n, n, n), order="F"), (0, 0, 0), fb, 1)
    orc.prolong(fb, 1, cb, 1, ec, uf, order=2)
    got = orc.unpack_valid(uf, (0, 0, 0), (n - 1,) * 3, fb, 1)
    x = [(np.arange(n) + 0.5) * h] * 3
    exp = a + b[0] * x[0][:, None, None] + b[1] * x[1][None, :, None] + b[2] * x[2][None, None, :]
    # interior fine cells (their coarse stencil never touches a boundary ghost)
    assert np.allclose(got[1:-1, 1:-1, 1:-1], exp[1:-1, 1:-1, 1:-1], rtol=0, atol=1e-14)


def test_piecewise_constant_then_restrict_is_identity(orc):
    fb = orc.chop((0, 0, 0), (11, 7, 7), 4)
    cb = [(tuple(x // 2 for x in lo), tuple(x // 2 for x in hi)) for lo, hi in fb]
    c = W.dyadic_codes((6, 4, 4), 12)
    ec = orc.pack(c, (0, 0, 0), cb, 1)
    uf = orc.pack(np.zeros((12, 8, 8), order="F"), (0, 0, 0), fb, 1)
    orc.prolong(fb, 1, cb, 1, ec, uf, order=1)
    fc = orc.restrict(fb, 1, cb, 1, uf)
    assert np.array_equal(orc.unpack_valid(fc, (0, 0, 0), (5, 3, 3), cb, 1), c)
