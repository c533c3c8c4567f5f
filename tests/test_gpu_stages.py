"""GPU parity of every stage kernel against the oracle, through the C ABI.

Ghost exchange, physical ghosts, restriction and prolongation move or combine
values in a fixed order, so they are compared bit for bit; the Gauss-Seidel
colour update and the residual follow the oracle's operation order (no FMA
contraction on either side) and are compared bit for bit as well.  The
bottom solve's CG reductions sum in a different order, so it is compared to
the oracle's bottom solve within the CG tolerance.  Shapes span several boxes
with ragged edges, negative lower corners and periodic self-images.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bx():
    import paper_2403_12179_amd as bx
    return bx


def make_ba(bx, dlo, dhi, mb, periodic):
    bc = tuple(bx.PERIODIC if p else bx.DIRICHLET0 for p in periodic)
    return bx.BoxArray.chop(dlo, dhi, mb, bc=bc)


def boxes_of(ba):
    return [(b.small, b.big) for b in ba.boxes]


FILL_CASES = [
    ((0, 0, 0), (15, 11, 7), 4, (1, 1, 1), 1, 1),
    ((0, 0, 0), (15, 11, 7), 4, (0, 0, 0), 1, 1),
    ((-6, -4, -2), (7, 5, 9), 4, (1, 0, 1), 1, 1),
    ((0, 0, 0), (5, 5, 5), 6, (1, 1, 1), 2, 1),
    ((0, 0, 0), (11, 11, 7), 4, (1, 0, 1), 2, 2),
    ((0, 0, 0), (1, 1, 1), 1, (1, 0, 1), 1, 1),
    ((0, 0, 0), (63, 63, 63), 32, (0, 0, 0), 1, 1),
]


@pytest.mark.parametrize("dlo,dhi,mb,per,ng,ncomp", FILL_CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fill_boundary_bitwise(bx, orc, dlo, dhi, mb, per, ng, ncomp, dtype):
    ba = make_ba(bx, dlo, dhi, mb, per)
    B = boxes_of(ba)
    shape = tuple(dhi[d] - dlo[d] + 1 for d in range(3))
    mf = bx.MultiFab(ba, ncomp=ncomp, nghost=ng, dtype=dtype)
    npdt = np.float64 if dtype == "f64" else np.float32
    comps = [W.dyadic_codes(shape, 100 + c) for c in range(ncomp)]
    packs = [orc.pack(g, dlo, B, ng, dtype=npdt) for g in comps]
    packed = []
    offs = [0] * ncomp
    for lo, hi in B:
        n = int(np.prod(orc.box_shape(lo, hi, ng)))
        for c in range(ncomp):
            packed.append(packs[c][offs[c]:offs[c] + n])
            offs[c] += n
    packed = np.ascontiguousarray(np.concatenate(packed))
    mf.from_packed(packed)
    mf.fill_boundary()
    orc.fill_boundary(dlo, dhi, per, B, ng, packed, ncomp=ncomp)
    assert np.array_equal(mf.to_packed(), packed, equal_nan=True)
    if dtype == "f64":
        mf.apply_domain_bc()
        orc.apply_bc(dlo, dhi, per, B, ng, packed, ncomp=ncomp)
        assert np.array_equal(mf.to_packed(), packed, equal_nan=True)
        mf.apply_domain_bc(odd=False)
        orc.apply_bc(dlo, dhi, per, B, ng, packed, ncomp=ncomp, odd=False)
        assert np.array_equal(mf.to_packed(), packed, equal_nan=True)


def test_fill_boundary_cross_and_holes(bx, orc):
    dlo, dhi = (0, 0, 0), (7, 7, 7)
    ba = bx.BoxArray.from_boxes(dlo, dhi, [((0, 0, 0), (3, 7, 7)), ((6, 0, 0), (7, 7, 7))], bc=(0, 0, 0))
    B = boxes_of(ba)
    mf = bx.MultiFab(ba)
    packed = orc.pack(W.dyadic_codes((8, 8, 8), 1), dlo, B, 1)
    mf.from_packed(packed)
    mf.fill_boundary()
    orc.fill_boundary(dlo, dhi, (1, 1, 1), B, 1, packed)
    assert np.array_equal(mf.to_packed(), packed, equal_nan=True)
    # faces only: edges and corners keep their NaN sentinels
    mf2 = bx.MultiFab(ba)
    p2 = orc.pack(W.dyadic_codes((8, 8, 8), 1), dlo, B, 1)
    mf2.from_packed(p2)
    mf2.fill_boundary(cross=True)
    v = mf2.array(0).cpu().numpy()
    assert np.isnan(v[0, 0, 1:-1]).all() and not np.isnan(v[0, 1:-1, 1:-1]).any()


STAGE_CASES = [
    ((0, 0, 0), (15, 15, 15), 8, (0, 0, 0)),
    ((0, 0, 0), (15, 15, 15), 8, (1, 1, 1)),
    ((-8, 0, -4), (7, 11, 11), 4, (1, 0, 1)),
    ((0, 0, 0), (31, 31, 31), 16, (0, 0, 0)),
]


def loaded(bx, orc, ba, dlo, glob, ghost=np.nan):
    mf = bx.MultiFab(ba)
    mf.from_packed(orc.pack(glob, dlo, boxes_of(ba), 1, ghost=ghost))
    return mf


@pytest.mark.parametrize("dlo,dhi,mb,per", STAGE_CASES)
@pytest.mark.parametrize("var", [False, True])
def test_gs_colour_bitwise(bx, orc, dlo, dhi, mb, per, var):
    ba = make_ba(bx, dlo, dhi, mb, per)
    B = boxes_of(ba)
    shape = tuple(dhi[d] - dlo[d] + 1 for d in range(3))
    h = 1.0 / shape[0]
    u0, f0 = W.uniform_rhs(shape, 1), W.uniform_rhs(shape, 2)
    beta = W.smooth_gaussian_beta(shape, 3) if var else None
    phi, rhs = loaded(bx, orc, ba, dlo, u0), loaded(bx, orc, ba, dlo, f0)
    bmf = loaded(bx, orc, ba, dlo, beta) if var else None
    U, F = orc.pack(u0, dlo, B, 1), orc.pack(f0, dlo, B, 1)
    for colour in (0, 1, 0):
        bx.gs_colour(phi, rhs, h, colour, beta=bmf)
        orc.fill_boundary(dlo, dhi, per, B, 1, U)
        orc.apply_bc(dlo, dhi, per, B, 1, U)
        orc.gs(dlo, dhi, per, B, h, colour, U, F, beta)
        got = phi.to_global()
        exp = orc.unpack_valid(U, dlo, dhi, B, 1)
        assert np.array_equal(got, exp), "colour %d" % colour


@pytest.mark.parametrize("dlo,dhi,mb,per", STAGE_CASES)
@pytest.mark.parametrize("var", [False, True])
def test_residual_bitwise(bx, orc, dlo, dhi, mb, per, var):
    ba = make_ba(bx, dlo, dhi, mb, per)
    B = boxes_of(ba)
    shape = tuple(dhi[d] - dlo[d] + 1 for d in range(3))
    h = 1.0 / shape[0]
    u0, f0 = W.uniform_rhs(shape, 5), W.uniform_rhs(shape, 6)
    beta = W.smooth_gaussian_beta(shape, 7) if var else None
    phi, rhs = loaded(bx, orc, ba, dlo, u0), loaded(bx, orc, ba, dlo, f0)
    bmf = loaded(bx, orc, ba, dlo, beta) if var else None
    r = bx.MultiFab(ba)
    rinf, rl2 = bx.residual(phi, rhs, h, r, beta=bmf)
    U, F = orc.pack(u0, dlo, B, 1), orc.pack(f0, dlo, B, 1)
    orc.fill_boundary(dlo, dhi, per, B, 1, U)
    orc.apply_bc(dlo, dhi, per, B, 1, U)
    R, oinf, ol2 = orc.residual(dlo, dhi, per, B, h, U, F, beta)
    assert np.array_equal(r.to_global(), orc.unpack_valid(R, dlo, dhi, B, 1))
    assert rinf == oinf
    assert abs(rl2 - ol2) <= 1e-13 * ol2


@pytest.mark.parametrize("dlo,dhi,mb", [((0, 0, 0), (15, 15, 15), 8), ((-8, 0, -4), (7, 11, 11), 4),
                                        ((0, 0, 0), (31, 15, 15), 16), ((0, 0, 0), (11, 7, 7), 4)])
def test_restrict_prolong_bitwise(bx, orc, dlo, dhi, mb):
    for per in [(0, 0, 0), (1, 1, 1), (1, 0, 1)]:
        ba = make_ba(bx, dlo, dhi, mb, per)
        B = boxes_of(ba)
        lv = ba.hierarchy()
        cdom, cboxes = lv[1]
        bc = tuple(bx.PERIODIC if p else bx.DIRICHLET0 for p in per)
        cba = bx.BoxArray.from_boxes(cdom.small, cdom.big, cboxes, bc=bc)
        CB = boxes_of(cba)
        shape = tuple(dhi[d] - dlo[d] + 1 for d in range(3))
        cshape = cdom.size
        g = W.uniform_rhs(shape, 11)
        fine = loaded(bx, orc, ba, dlo, g)
        coarse = bx.MultiFab(cba).set_val(0.0)
        bx.restrict(fine, coarse)
        exp = orc.restrict(B, 1, CB, 1, orc.pack(g, dlo, B, 1))
        assert np.array_equal(coarse.to_global(), orc.unpack_valid(exp, cdom.small, cdom.big, CB, 1))
        # prolongation
        e = W.uniform_rhs(cshape, 12)
        for order in (1, 2):
            cmf = loaded(bx, orc, cba, cdom.small, e)
            fmf = loaded(bx, orc, ba, dlo, g)
            bx.prolong_add(cmf, fmf, order=order)
            E = orc.pack(e, cdom.small, CB, 1)
            orc.fill_boundary(cdom.small, cdom.big, per, CB, 1, E)
            orc.apply_bc(cdom.small, cdom.big, per, CB, 1, E)
            U = orc.pack(g, dlo, B, 1)
            orc.prolong(B, 1, CB, 1, E, U, order=order)
            assert np.array_equal(fmf.to_global(), orc.unpack_valid(U, dlo, dhi, B, 1)), (per, order)


@pytest.mark.parametrize("shape,per", [((2, 2, 2), (0, 0, 0)), ((3, 3, 3), (1, 1, 1)), ((15, 15, 15), (0, 0, 0)),
                                       ((7, 5, 3), (1, 0, 1)), ((16, 16, 16), (1, 1, 1))])
def test_bottom_cg(bx, orc, shape, per):
    dlo, dhi = (0, 0, 0), tuple(x - 1 for x in shape)
    ba = make_ba(bx, dlo, dhi, 8, per)
    h = 1.0 / shape[0]
    f = W.uniform_rhs(shape, 13, mean_zero=(per == (1, 1, 1)))
    phi = bx.MultiFab(ba).set_val(0.0)
    rhs = loaded(bx, orc, ba, dlo, f)
    it = bx.bottom_solve(phi, rhs, h)
    u_o, it_o = orc.bottom(dlo, dhi, per, h, f)
    got = phi.to_global()
    assert np.max(np.abs(got - u_o)) <= 1e-10 * np.max(np.abs(u_o))
    assert abs(it - it_o) <= 2
    Lu = orc.apply_op(dlo, dhi, per, h, got)
    fp = f - f.mean() if per == (1, 1, 1) else f
    assert np.max(np.abs(fp - Lu)) <= 1e-10 * np.max(np.abs(f))


def test_multifab_copy_host_roundtrip(bx):
    """bxmg_multifab_copy_host writes exactly the valid cells of one
    component (ghosts and other components keep their values) and reads them
    back in the global F-order layout."""
    ba = bx.BoxArray.chop((-4, 0, 2), (11, 9, 13), 8, bc=(bx.PERIODIC, bx.DIRICHLET0, bx.PERIODIC))
    shape = ba.domain.size
    for dtype, npdt in (("f64", np.float64), ("f32", np.float32)):
        mf = bx.MultiFab(ba, ncomp=2, nghost=2, dtype=dtype).set_val(-7.0)
        g = np.asfortranarray(W.dyadic_codes(shape, 3).astype(npdt))
        mf.copy_host(g, to_device=True, comp=1)
        packed = mf.to_packed()
        assert np.array_equal(mf.to_global(comp=1), g)
        assert np.all(mf.to_global(comp=0) == -7.0)
        n_valid = int(np.prod(shape))
        assert np.count_nonzero(packed != -7.0) == n_valid  # ghosts and component 0 untouched
        back = np.asfortranarray(np.zeros(shape, npdt))
        mf.copy_host(back, to_device=False, comp=1)
        assert np.array_equal(back, g)


def test_library_owned_multifab_stream_ordered_release(bx):
    """A MultiFab whose slab the library allocates (device_buf = NULL) takes
    and returns data; releasing it right after enqueueing ghost exchanges on
    the context's stream, without waiting, leaves later allocations and
    their data intact."""
    import ctypes as C
    lib, ctx = bx.lib(), bx.default_context()
    ba = bx.BoxArray.chop((0, 0, 0), (31, 23, 15), 8, bc=(bx.PERIODIC, bx.DIRICHLET0, bx.PERIODIC))
    shape = ba.domain.size
    for it in range(4):
        g = np.asfortranarray(W.dyadic_codes(shape, 50 + it))
        h = C.c_void_p()
        bx._lib.check(lib.bxmg_alloc_multifab(ctx._h, ba._h, 2, 1, 0, None, C.byref(h)))
        bx._lib.check(lib.bxmg_multifab_copy_host(h, 1, g.ctypes.data, 1, None))
        for _ in range(3):
            bx._lib.check(lib.bxmg_fill_boundary(h, 0, 2, 0, None))
        back = np.asfortranarray(np.zeros(shape))
        bx._lib.check(lib.bxmg_multifab_copy_host(h, 0, back.ctypes.data, 1, None))
        assert np.array_equal(back, g)
        for _ in range(3):
            bx._lib.check(lib.bxmg_fill_boundary(h, 0, 2, 0, None))
        lib.bxmg_multifab_release(h)  # exchanges may still be queued
    import torch
    torch.cuda.synchronize()
