"""Oracle pins for the two-level composite solve (a coarse level over the
domain, a fine level of refinement ratio 2 over a union of boxes; the
paper's block-structured AMR hierarchy, Sections 1 and 2).

* The composite operator is exact on linear and harmonic quadratic fields
  (the coarse-fine ghost interpolation is quadratic in all three
  directions, the fine stencil and the flux-matched coarse faces are exact
  on quadratics), at every fine cell and every uncovered coarse cell away
  from the domain boundary -- for a single refined cube and for an L of
  abutting boxes plus a detached one.
* Conservation: on a periodic domain, h0^3 sum Lc + h1^3 sum Lf is zero for
  any field (the coarse flux across a coarse-fine face is the mean of the
  fine fluxes through it).
* With no fine boxes the composite solve is the plain single-level solve.
* On 8^3 + one fine box the solve matches numpy's dense solve of the
  composite system assembled column by column.
* A manufactured sine solution converges at second order; the cycle
  contracts at an h-independent rate; covered coarse cells hold the mean of
  their children; unsupported layouts are refused.
"""
import numpy as np
import pytest

import workloads as W


def centres(n, h):
    return (np.arange(n) + 0.5) * h


def field(n, h, fn):
    x = centres(n, h)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    return fn(X, Y, Z)


def covered_mask(n, fb):
    m = np.zeros((n, n, n), bool)
    for lo, hi in fb:
        m[lo[0] // 2:hi[0] // 2 + 1, lo[1] // 2:hi[1] // 2 + 1, lo[2] // 2:hi[2] // 2 + 1] = True
    return m


QUADS = [
    lambda X, Y, Z: 1.0 + 2 * X - 3 * Y + 0.5 * Z,
    lambda X, Y, Z: X * X - Y * Y,
    lambda X, Y, Z: X * X + Y * Y - 2 * Z * Z,
    lambda X, Y, Z: X * Y,
    lambda X, Y, Z: Y * Z - 2 * X * Z,
]


@pytest.mark.parametrize("kind", ["centre", "lshape"])
@pytest.mark.parametrize("q", range(len(QUADS)))
def test_exact_on_harmonic_quadratics(orc, kind, q):
    n = 16
    h = 1.0 / n
    cb, fb = W.composite_layout(n, kind, max_box=8)
    fn = QUADS[q]
    Lc, Lf = orc.composite_apply(n, (0, 0, 0), cb, fb, h, field(n, h, fn), field(2 * n, h / 2, fn))
    inner = np.zeros((n, n, n), bool)
    inner[1:-1, 1:-1, 1:-1] = True
    cov = covered_mask(n, fb)
    scale = 1.0 / h ** 2
    assert np.abs(Lc[inner & ~cov]).max() < 1e-12 * scale
    assert np.all(Lc[cov] == 0.0)
    fm = W.fine_mask(n, fb)
    assert np.abs(Lf[fm]).max() < 1e-12 * scale
    assert np.all(Lf[~fm] == 0.0)


def test_not_exact_on_cubics(orc):
    """The exactness above is not vacuous: a cubic leaves an O(h) error at
    the coarse-fine boundary only."""
    n = 16
    h = 1.0 / n
    cb, fb = W.composite_layout(n, "centre", max_box=8)
    fn = lambda X, Y, Z: X ** 3 - 3 * X * Y * Y
    Lc, Lf = orc.composite_apply(n, (0, 0, 0), cb, fb, h, field(n, h, fn), field(2 * n, h / 2, fn))
    fm = W.fine_mask(n, fb)
    assert np.abs(Lf[fm]).max() > 1e-3


@pytest.mark.parametrize("kind", ["centre", "lshape"])
def test_conservation_periodic(orc, kind):
    n = 16
    h = 1.0 / n
    cb, fb = W.composite_layout(n, kind, max_box=8)
    rng = np.random.default_rng(7)
    uc = rng.standard_normal((n, n, n))
    uf = rng.standard_normal((2 * n,) * 3)
    Lc, Lf = orc.composite_apply(n, (1, 1, 1), cb, fb, h, uc, uf)
    tot = h ** 3 * Lc.sum() + (h / 2) ** 3 * Lf.sum()
    mag = h ** 3 * np.abs(Lc).sum() + (h / 2) ** 3 * np.abs(Lf).sum()
    assert abs(tot) < 1e-13 * mag


def test_no_fine_is_plain_solve(orc):
    n = 16
    cb = W.chop_boxes(n, 8)
    f = W.uniform_rhs((n, n, n), seed=3)
    uc, uf, info = orc.composite_solve(n, (0, 0, 0), cb, [], f, np.zeros((2 * n,) * 3), rel_tol=1e-12)
    u, inf2 = orc.solve((0, 0, 0), (n - 1,) * 3, (0, 0, 0), cb, f, rel_tol=1e-12)
    assert info["status"] == 0 and inf2["status"] == 0
    assert np.abs(uc - u).max() < 1e-10 * np.abs(u).max()
    assert np.all(uf == 0.0)


def test_dense_composite_system(orc):
    """Assemble the composite operator column by column over the unknowns
    (uncovered coarse cells, fine cells) and solve with numpy."""
    n = 8
    h = 1.0 / n
    cb = W.chop_boxes(n, 8)
    fb = [((4, 4, 4), (11, 11, 11))]
    cov = covered_mask(n, fb)
    fm = W.fine_mask(n, fb)
    ic = np.flatnonzero(~cov.ravel(order="F"))
    jf = np.flatnonzero(fm.ravel(order="F"))
    N = ic.size + jf.size
    A = np.zeros((N, N))
    for col in range(N):
        uc = np.zeros(n ** 3)
        uf = np.zeros((2 * n) ** 3)
        if col < ic.size:
            uc[ic[col]] = 1.0
        else:
            uf[jf[col - ic.size]] = 1.0
        Lc, Lf = orc.composite_apply(n, (0, 0, 0), cb, fb, h, uc.reshape((n,) * 3, order="F"),
                                     uf.reshape((2 * n,) * 3, order="F"))
        A[:, col] = np.concatenate([Lc.ravel(order="F")[ic], Lf.ravel(order="F")[jf]])
    rng = np.random.default_rng(11)
    fc = rng.uniform(-1, 1, (n, n, n))
    ff = rng.uniform(-1, 1, (2 * n,) * 3)
    b = np.concatenate([fc.ravel(order="F")[ic], ff.ravel(order="F")[jf]])
    x = np.linalg.solve(A, b)
    uc, uf, info = orc.composite_solve(n, (0, 0, 0), cb, fb, fc, ff, rel_tol=1e-13)
    assert info["status"] == 0
    got = np.concatenate([uc.ravel(order="F")[ic], uf.ravel(order="F")[jf]])
    assert np.abs(got - x).max() < 1e-9 * np.abs(x).max()


def manufactured(orc, n, kind="centre"):
    h = 1.0 / n
    cb, fb = W.composite_layout(n, kind, max_box=16)
    ex = lambda X, Y, Z: np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)
    fc = -3 * np.pi ** 2 * field(n, h, ex)
    ff = -3 * np.pi ** 2 * field(2 * n, h / 2, ex)
    uc, uf, info = orc.composite_solve(n, (0, 0, 0), cb, fb, fc, ff, rel_tol=1e-11)
    assert info["status"] == 0
    cov = covered_mask(n, fb)
    fm = W.fine_mask(n, fb)
    ec = np.abs(uc - field(n, h, ex))[~cov].max()
    ef = np.abs(uf - field(2 * n, h / 2, ex))[fm].max()
    return max(ec, ef), info, uc, uf, fb


def test_second_order_and_contraction(orc):
    e16, i16, _, _, _ = manufactured(orc, 16)
    e32, i32, _, _, _ = manufactured(orc, 32)
    assert 3.5 < e16 / e32 < 4.6
    for info in (i16, i32):
        hist = info["hist"]
        rates = [hist[k + 1] / hist[k] for k in range(1, min(len(hist) - 1, 6))]
        assert max(rates) < 0.2
    assert abs(i16["cycles"] - i32["cycles"]) <= 1


def test_covered_cells_hold_mean_of_children(orc):
    n = 16
    _, _, uc, uf, fb = manufactured(orc, n, "lshape")
    cov = covered_mask(n, fb)
    mean = uf.reshape(n, 2, n, 2, n, 2, order="C").mean(axis=(1, 3, 5))
    assert np.abs(uc[cov] - mean[cov]).max() < 1e-15 * np.abs(uf).max() * 8


def test_periodic_compatible_solve(orc):
    n = 16
    h = 1.0 / n
    cb, fb = W.composite_layout(n, "lshape")
    rng = np.random.default_rng(5)
    cov = covered_mask(n, fb)
    fm = W.fine_mask(n, fb)
    fc = rng.standard_normal((n, n, n))
    ff = rng.standard_normal((2 * n,) * 3)
    fc[cov] = 0.0
    ff[~fm] = 0.0
    tot = h ** 3 * fc.sum() + (h / 2) ** 3 * ff.sum()
    vol = h ** 3 * (~cov).sum() + (h / 2) ** 3 * fm.sum()
    fc[~cov] -= tot / vol
    ff[fm] -= tot / vol
    uc, uf, info = orc.composite_solve(n, (1, 1, 1), cb, fb, fc, ff, rel_tol=1e-10)
    assert info["status"] == 0 and info["cycles"] < 20
    Lc, Lf = orc.composite_apply(n, (1, 1, 1), cb, fb, h, uc, uf)
    assert np.abs(Lc - fc)[~cov].max() < 1e-9 * np.abs(fc).max()
    assert np.abs(Lf - ff)[fm].max() < 1e-9 * np.abs(ff).max()


@pytest.mark.parametrize("bad", [
    [((2, 4, 4), (11, 11, 11))],           # within 2 coarse cells of the boundary
    [((5, 4, 4), (12, 11, 11))],           # not aligned to coarse cells
    [((4, 4, 4), (11, 11, 11)), ((10, 4, 4), (15, 11, 11))],  # overlapping
])
def test_layout_refused(orc, bad):
    n = 16
    with pytest.raises(ValueError):
        orc.composite_apply(n, (0, 0, 0), W.chop_boxes(n, 8), bad, 1.0 / n, np.zeros((n,) * 3),
                            np.zeros((2 * n,) * 3))
