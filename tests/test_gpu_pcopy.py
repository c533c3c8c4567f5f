"""GPU ParallelCopy (bxmg_parallel_copy) bitwise against the oracle's, for
several pairs of decompositions, ghost widths, component ranges, source
holes and both precisions (the fields are dyadic codes, exact in FP32)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bx():
    import paper_2403_12179_amd as bx
    return bx


def packed_multi(orc, comps, dom_lo, boxes, ng, fill=np.nan):
    parts = []
    packs = [orc.pack(c, dom_lo, boxes, ng, ghost=fill) for c in comps]
    offs = [0] * len(comps)
    for lo, hi in boxes:
        n = int(np.prod(orc.box_shape(lo, hi, ng)))
        for c in range(len(comps)):
            parts.append(packs[c][offs[c]:offs[c] + n])
            offs[c] += n
    return np.concatenate(parts)


CASES = [
    ((0, 0, 0), (15, 11, 9), (1, 1, 1), 8, 5, 1, 1),
    ((-4, 0, 2), (11, 9, 13), (1, 0, 1), 6, 4, 2, 2),
    ((0, 0, 0), (12, 12, 12), (0, 0, 0), 7, 13, 1, 0),
    ((0, 0, 0), (63, 63, 63), (1, 1, 1), 32, 16, 1, 1),
]


@pytest.mark.parametrize("dlo,dhi,per,mb_src,mb_dst,ng,ngc", CASES)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_parallel_copy_bitwise(bx, orc, dlo, dhi, per, mb_src, mb_dst, ng, ngc, dtype):
    shape = tuple(dhi[d] - dlo[d] + 1 for d in range(3))
    bc = tuple(bx.PERIODIC if p else bx.DIRICHLET0 for p in per)
    bs = bx.BoxArray.chop(dlo, dhi, mb_src, bc=bc)
    bd = bx.BoxArray.chop(dlo, dhi, mb_dst, bc=bc)
    sb = [(b.small, b.big) for b in bs.boxes]
    db = [(b.small, b.big) for b in bd.boxes]
    G0, G1 = W.dyadic_codes(shape, 21), W.dyadic_codes(shape, 22)
    src = packed_multi(orc, [G0, G1], dlo, sb, 1)
    dst = packed_multi(orc, [np.full(shape, np.nan)] * 3, dlo, db, ng)
    want = orc.parallel_copy(dlo, dhi, per, db, ng, dst, sb, 1, src, ncomp=2, dst_ncomp=3, src_ncomp=2, dcomp=1,
                             scomp=0, copy_ng=ngc)
    npdt = np.float64 if dtype == "f64" else np.float32
    ms = bx.MultiFab(bs, ncomp=2, nghost=1, dtype=dtype)
    md = bx.MultiFab(bd, ncomp=3, nghost=ng, dtype=dtype)
    ms.from_packed(src.astype(npdt))
    md.from_packed(dst.astype(npdt))
    md.parallel_copy(ms, scomp=0, dcomp=1, ncomp=2, nghost=ngc)
    assert np.array_equal(md.to_packed(), want.astype(npdt), equal_nan=True)


def test_parallel_copy_from_holes_and_errors(bx, orc):
    import ctypes as C
    dlo, dhi = (0, 0, 0), (11, 11, 11)
    src_boxes = [((0, 0, 0), (5, 11, 11)), ((8, 0, 0), (11, 5, 11))]
    bs = bx.BoxArray.from_boxes(dlo, dhi, src_boxes, bc=(bx.PERIODIC, bx.PERIODIC, bx.DIRICHLET0))
    bd = bx.BoxArray.chop(dlo, dhi, 4, bc=(bx.PERIODIC, bx.PERIODIC, bx.DIRICHLET0))
    db = [(b.small, b.big) for b in bd.boxes]
    G = W.dyadic_codes((12, 12, 12), 23)
    src = orc.pack(G, dlo, src_boxes, 1)
    dst = orc.pack(np.full((12, 12, 12), -7.0), dlo, db, 1, ghost=-7.0)
    want = orc.parallel_copy(dlo, dhi, (1, 1, 0), db, 1, dst, src_boxes, 1, src, copy_ng=1)
    ms, md = bx.MultiFab(bs), bx.MultiFab(bd)
    ms.from_packed(src)
    md.from_packed(dst)
    md.parallel_copy(ms, nghost=1)
    assert np.array_equal(md.to_packed(), want)
    lib = bx.lib()
    other = bx.BoxArray.chop(dlo, dhi, 4)  # Dirichlet everywhere: another boundary set
    mo = bx.MultiFab(other)
    assert lib.bxmg_parallel_copy(mo._h, 0, ms._h, 0, 1, 0, None) == -1
    assert lib.bxmg_parallel_copy(md._h, 0, ms._h, 0, 1, 2, None) == -1  # wider than md's ghosts
    assert lib.bxmg_parallel_copy(md._h, 0, ms._h, 0, 2, 0, None) == -1  # components
