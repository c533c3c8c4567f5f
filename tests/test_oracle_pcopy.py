"""Oracle pins for ParallelCopy (copies between two box decompositions of
one domain): the result is checked against numpy's own construction of the
expected destination from the global field -- np.pad with 'wrap' in the
periodic directions, untouched sentinels beyond non-periodic faces and over
holes in the source decomposition -- for several decompositions, ghost
widths and component ranges."""
import numpy as np
import pytest

import workloads as W


def expected(G, dom_lo, per, dst_boxes, ng_alloc, ng_copy, ncomp_d, dcomp, comps, covered, fill=np.nan):
    """Packed destination after the copy, from the global source fields."""
    pads = [(ng_alloc, ng_alloc)] * 3
    out = []
    for lo, hi in dst_boxes:
        shape = tuple(hi[d] - lo[d] + 1 + 2 * ng_alloc for d in range(3))
        for c in range(ncomp_d):
            a = np.full(shape, fill, order="F")
            if dcomp <= c < dcomp + len(comps):
                src = comps[c - dcomp]
                # global field padded by ng_alloc: wrap where periodic, NaN elsewhere
                P = src
                for d in range(3):
                    w = [(0, 0)] * 3
                    w[d] = pads[d]
                    P = np.pad(P, w, mode="wrap") if per[d] else np.pad(P, w, mode="constant", constant_values=np.nan)
                C = covered
                for d in range(3):
                    w = [(0, 0)] * 3
                    w[d] = pads[d]
                    C = np.pad(C, w, mode="wrap") if per[d] else np.pad(C, w, mode="constant", constant_values=False)
                s = tuple(slice(lo[d] - dom_lo[d], hi[d] - dom_lo[d] + 1 + 2 * ng_alloc) for d in range(3))
                vals, cov = P[s], C[s]
                inner = np.zeros(shape, bool)
                g0 = ng_alloc - ng_copy
                inner[g0:shape[0] - g0, g0:shape[1] - g0, g0:shape[2] - g0] = True
                take = inner & cov
                a[take] = vals[take]
            out.append(a.ravel(order="F"))
    return np.concatenate(out)


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
    ((0, 0, 0), (12, 12, 12), (0, 0, 0), 7, 13, 1, 1),
    ((0, 0, 0), (7, 7, 7), (0, 1, 0), 4, 3, 2, 1),
]


@pytest.mark.parametrize("dlo,dhi,per,mb_src,mb_dst,ng_alloc,ng_copy", CASES)
def test_parallel_copy_against_numpy(orc, dlo, dhi, per, mb_src, mb_dst, ng_alloc, ng_copy):
    shape = tuple(dhi[d] - dlo[d] + 1 for d in range(3))
    src_boxes = orc.chop(dlo, dhi, mb_src)
    dst_boxes = orc.chop(dlo, dhi, mb_dst)
    G0, G1 = W.dyadic_codes(shape, 11), W.dyadic_codes(shape, 12)
    src = packed_multi(orc, [G0, G1], dlo, src_boxes, 1)
    dst = packed_multi(orc, [np.full(shape, np.nan)] * 3, dlo, dst_boxes, ng_alloc)
    out = orc.parallel_copy(dlo, dhi, per, dst_boxes, ng_alloc, dst, src_boxes, 1, src, ncomp=2, dst_ncomp=3,
                            src_ncomp=2, dcomp=1, scomp=0, copy_ng=ng_copy)
    want = expected([G0, G1], dlo, per, dst_boxes, ng_alloc, ng_copy, 3, 1, [G0, G1], np.ones(shape, bool))
    assert np.array_equal(out, want, equal_nan=True)


def test_parallel_copy_from_boxes_with_holes(orc):
    dlo, dhi, per = (0, 0, 0), (11, 11, 11), (1, 1, 0)
    shape = (12, 12, 12)
    src_boxes = [((0, 0, 0), (5, 11, 11)), ((8, 0, 0), (11, 5, 11))]  # cells x in 6..7, and y >= 6 for x >= 8: holes
    covered = np.zeros(shape, bool)
    for lo, hi in src_boxes:
        covered[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1] = True
    G = W.dyadic_codes(shape, 13)
    src = orc.pack(G, dlo, src_boxes, 0)
    dst_boxes = orc.chop(dlo, dhi, 4)
    dst = orc.pack(np.full(shape, -7.0), dlo, dst_boxes, 1, ghost=-7.0)
    out = orc.parallel_copy(dlo, dhi, per, dst_boxes, 1, dst, src_boxes, 0, src, copy_ng=1)
    want = expected([G], dlo, per, dst_boxes, 1, 1, 1, 0, [G], covered, fill=-7.0)
    assert np.array_equal(out, want)
