"""GPU two-level composite solve (bxmg_composite_solve) against the oracle's
composite solve: element by element after a fixed number of cycles (both
sides run the same iteration, so the iterates agree to rounding), converged
solutions and residual histories, a periodic problem (solutions agree up to
the constant the singular problem leaves free), layouts of one refined cube
in many boxes and of an L of abutting boxes plus a detached one, ragged
coarse boxes, and at the full size (512^3-cell fine domain, 256^3 refined
cells in 512 boxes) the oracle's composite residual of the GPU's solution.

Tolerances: a fixed-cycle iterate differs from the oracle's only by rounding
in the ~10^2 operations per cell and cycle, amplified at most by the
cycle's contraction (< 1), so 1e-9 of max|u| is loose; converged solutions
both meet |r| <= 1e-10 |f|, and the composite operator's inverse is O(1) in
these units, so they agree to a few 1e-9 of max|u|."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bx():
    import paper_2403_12179_amd as bx
    return bx


def cov_mask(n, fb):
    m = np.zeros((n, n, n), bool)
    for lo, hi in fb:
        m[lo[0] // 2:hi[0] // 2 + 1, lo[1] // 2:hi[1] // 2 + 1, lo[2] // 2:hi[2] // 2 + 1] = True
    return m


def gpu_solve(bx, n, per, cb, fb, fc, ff, ngf=1, check_ghosts=False, **params):
    bc = tuple(bx.PERIODIC if p else bx.DIRICHLET0 for p in per)
    cba = bx.BoxArray.from_boxes((0, 0, 0), (n - 1,) * 3, cb, bc=bc)
    fba = bx.BoxArray.from_boxes((0, 0, 0), (2 * n - 1,) * 3, fb, bc=bc)
    pc = bx.MultiFab(cba, nghost=1).set_val(np.nan)  # contents on entry are ignored
    rc = bx.MultiFab(cba, nghost=0).from_global(np.asfortranarray(fc))
    pf = bx.MultiFab(fba, nghost=ngf).set_val(np.nan)
    rf = bx.MultiFab(fba, nghost=2).from_global(np.asfortranarray(ff), ghost=np.nan)
    res = bx.composite_solve(pc, rc, pf, rf, **params)
    if check_ghosts:  # the fine solution's ghost cells are left alone (NaN), its valid cells written
        packed = pf.to_packed()
        valid = sum((hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1) for lo, hi in fb)
        assert np.isnan(packed).sum() == packed.size - valid
    return pc.to_global(), pf.to_global(), res


def rhs(n, fb, seed):
    fc = W.uniform_rhs((n, n, n), seed=seed)
    ff = W.uniform_rhs((2 * n,) * 3, seed=seed + 1)
    return fc, ff


CASES = [
    # n, kind, fine max box, coarse box edge
    (16, "lshape", 8, 8),
    (32, "centre", 16, 16),
    (32, "centre", 8, 12),   # ragged coarse boxes
    (32, "holed", 8, 16),    # 63 abutting fine boxes, not merged: ghosts copied between them
]


@pytest.mark.parametrize("n,kind,fmax,cmax", CASES)
def test_fixed_cycles_elementwise(bx, orc, n, kind, fmax, cmax):
    _, fb = W.composite_layout(n, kind, max_box=fmax)
    cb = W.chop_boxes(n, cmax)
    fc, ff = rhs(n, fb, 31)
    print("composite fixed cycles", n, kind, len(fb), "fine boxes", flush=True)
    uc_o, uf_o, io = orc.composite_solve(n, (0, 0, 0), cb, fb, fc, ff, fixed_cycles=4)
    uc_g, uf_g, ig = gpu_solve(bx, n, (0, 0, 0), cb, fb, fc, ff, check_ghosts=True, fixed_cycles=4)
    assert ig.status == 0 and ig.cycles == 4 == io["cycles"]
    scale = max(np.abs(uc_o).max(), np.abs(uf_o).max())
    fm = W.fine_mask(n, fb)
    assert np.abs(uc_g - uc_o).max() <= 1e-9 * scale
    assert np.abs(uf_g[fm] - uf_o[fm]).max() <= 1e-9 * scale
    assert np.all(np.isnan(uf_g[~fm]))
    np.testing.assert_allclose(ig.hist, io["hist"], rtol=1e-7)
    np.testing.assert_allclose(ig.hist_l2, io["hist_l2"], rtol=1e-7)
    assert ig.f_inf == pytest.approx(io["f_inf"], rel=1e-15)


@pytest.mark.parametrize("per", [(1, 0, 0), (0, 1, 1)])
def test_mixed_boundaries_elementwise(bx, orc, per):
    """Periodic in some directions, Dirichlet in the others (non-singular)."""
    n = 16
    _, fb = W.composite_layout(n, "lshape")
    cb = W.chop_boxes(n, 8)
    fc, ff = rhs(n, fb, 91)
    uc_o, uf_o, io = orc.composite_solve(n, per, cb, fb, fc, ff, fixed_cycles=3)
    uc_g, uf_g, ig = gpu_solve(bx, n, per, cb, fb, fc, ff, fixed_cycles=3)
    assert ig.status == 0 and io["status"] == 0
    scale = max(np.abs(uc_o).max(), np.abs(uf_o).max())
    fm = W.fine_mask(n, fb)
    assert np.abs(uc_g - uc_o).max() <= 1e-9 * scale
    assert np.abs(uf_g[fm] - uf_o[fm]).max() <= 1e-9 * scale
    np.testing.assert_allclose(ig.hist, io["hist"], rtol=1e-7)


@pytest.mark.parametrize("n,kind,fmax,cmax", CASES[:2])
def test_converged(bx, orc, n, kind, fmax, cmax):
    _, fb = W.composite_layout(n, kind, max_box=fmax)
    cb = W.chop_boxes(n, cmax)
    fc, ff = rhs(n, fb, 41)
    uc_o, uf_o, io = orc.composite_solve(n, (0, 0, 0), cb, fb, fc, ff, rel_tol=1e-10)
    uc_g, uf_g, ig = gpu_solve(bx, n, (0, 0, 0), cb, fb, fc, ff, rel_tol=1e-10)
    assert ig.status == 0 and io["status"] == 0
    assert abs(ig.cycles - io["cycles"]) <= 1
    assert ig.rel_resid_inf <= 1e-10
    scale = max(np.abs(uc_o).max(), np.abs(uf_o).max())
    fm = W.fine_mask(n, fb)
    assert np.abs(uc_g - uc_o).max() <= 5e-9 * scale
    assert np.abs(uf_g[fm] - uf_o[fm]).max() <= 5e-9 * scale
    # covered coarse cells hold the mean of their children
    cov = cov_mask(n, fb)
    mean = np.where(fm, uf_g, 0.0).reshape(n, 2, n, 2, n, 2).mean(axis=(1, 3, 5))
    assert np.abs(uc_g[cov] - mean[cov]).max() <= 1e-14 * scale


def test_periodic_up_to_constant(bx, orc):
    n = 16
    h = 1.0 / n
    cb, fb = W.composite_layout(n, "lshape")
    cov = cov_mask(n, fb)
    fm = W.fine_mask(n, fb)
    fc, ff = rhs(n, fb, 51)
    fc[cov] = 0.0
    ff[~fm] = 0.0
    tot = h ** 3 * fc.sum() + (h / 2) ** 3 * ff.sum()
    vol = h ** 3 * (~cov).sum() + (h / 2) ** 3 * fm.sum()
    fc[~cov] -= tot / vol
    ff[fm] -= tot / vol
    uc_o, uf_o, io = orc.composite_solve(n, (1, 1, 1), cb, fb, fc, ff, rel_tol=1e-10)
    uc_g, uf_g, ig = gpu_solve(bx, n, (1, 1, 1), cb, fb, fc, ff, rel_tol=1e-10)
    assert ig.status == 0 and io["status"] == 0

    def centred(uc, uf):
        m = (h ** 3 * uc[~cov].sum() + (h / 2) ** 3 * uf[fm].sum()) / vol
        return uc - m, uf - m

    a_c, a_f = centred(uc_o, uf_o)
    b_c, b_f = centred(uc_g, uf_g)
    scale = max(np.abs(a_c).max(), np.abs(a_f[fm]).max())
    assert np.abs(a_c - b_c).max() <= 5e-9 * scale
    assert np.abs(a_f[fm] - b_f[fm]).max() <= 5e-9 * scale


def test_repeat_and_relayout(bx, orc):
    """Cached per-layout state: a second layout, then the first again (and
    fine solution fields with 0, 2 and 1 ghost layers)."""
    n = 16
    for kind, ngf in (("lshape", 0), ("centre", 2), ("lshape", 1)):
        _, fb = W.composite_layout(n, kind, max_box=8)
        cb = W.chop_boxes(n, 8)
        fc, ff = rhs(n, fb, 61)
        uc_o, uf_o, io = orc.composite_solve(n, (0, 0, 0), cb, fb, fc, ff, fixed_cycles=2)
        uc_g, uf_g, ig = gpu_solve(bx, n, (0, 0, 0), cb, fb, fc, ff, ngf=ngf, fixed_cycles=2)
        scale = max(np.abs(uc_o).max(), np.abs(uf_o).max())
        fm = W.fine_mask(n, fb)
        assert np.abs(uc_g - uc_o).max() <= 1e-9 * scale
        assert np.abs(uf_g[fm] - uf_o[fm]).max() <= 1e-9 * scale


def test_zero_rhs(bx):
    n = 16
    cb, fb = W.composite_layout(n, "centre", max_box=8)
    uc, uf, res = gpu_solve(bx, n, (0, 0, 0), cb, fb, np.zeros((n,) * 3), np.zeros((2 * n,) * 3))
    assert res.status == 0 and res.cycles == 0
    assert np.all(uc == 0.0) and np.all(uf[W.fine_mask(n, fb)] == 0.0)


@pytest.mark.parametrize("bad", [
    [((2, 4, 4), (11, 11, 11))],    # within 2 coarse cells of the boundary
    [((5, 4, 4), (12, 11, 11))],    # not whole coarse cells
])
def test_layout_refused(bx, bad):
    n = 16
    with pytest.raises(bx.BxmgError):
        gpu_solve(bx, n, (0, 0, 0), W.chop_boxes(n, 8), bad, np.zeros((n,) * 3), np.zeros((2 * n,) * 3))


def test_full_size_residual_by_oracle(bx, orc):
    """256^3 coarse cells, the central half refined (256^3 fine cells in 512
    boxes of 32^3): the oracle's composite operator applied to the GPU's
    solution leaves |f - L u| <= rel_tol |f| (up to rounding)."""
    n = 256
    cb, fb = W.composite_layout(n, "centre", max_box=32)
    assert len(fb) == 512
    fc = W.uniform_rhs((n, n, n), seed=71)
    ff = np.zeros((2 * n,) * 3, order="F")
    fm = W.fine_mask(n, fb)
    lo, hi = n // 2, 3 * n // 2
    ff[lo:hi, lo:hi, lo:hi] = W.uniform_rhs((n, n, n), seed=72)
    print("composite full size: GPU solve", flush=True)
    uc, uf, res = gpu_solve(bx, n, (0, 0, 0), cb, fb, fc, ff, rel_tol=1e-10)
    assert res.status == 0 and res.rel_resid_inf <= 1e-10
    assert res.cycles <= 14
    print("composite full size: oracle residual", flush=True)
    uf = np.where(fm, uf, 0.0)
    Lc, Lf = orc.composite_apply(n, (0, 0, 0), cb, fb, 1.0 / n, uc, uf)
    cov = cov_mask(n, fb)
    fnorm = max(np.abs(fc[~cov]).max(), np.abs(ff[fm]).max())
    r = max(np.abs(fc - Lc)[~cov].max(), np.abs(ff - Lf)[fm].max())
    assert r <= 1.5e-10 * fnorm
    assert res.rel_resid_inf == pytest.approx(r / fnorm, rel=0.2, abs=1e-13)
