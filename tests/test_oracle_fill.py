"""Oracle pins: FillBoundary (ghost cell exchange, paper Section 2) and the
homogeneous Dirichlet ghost rule.

The expected ghost values come from numpy.pad on the global array: 'wrap' for
periodic directions; for a Dirichlet direction FillBoundary leaves the ghost
untouched (NaN sentinel survives) and the boundary condition then sets
-(mirror), i.e. numpy.pad 'symmetric' with the padded slab negated.  Inputs
are exactly representable codes, so equality is bitwise.
"""
import numpy as np
import pytest

import workloads as W


def padded_expect(glob, periodic, ng, bc):
    """Global array padded by ng: wrap on periodic axes; on the others NaN
    (fill only) or -(mirror) (fill then Dirichlet)."""
    a = glob.copy()
    for d in range(3):
        pw = [(0, 0)] * 3
        pw[d] = (ng, ng)
        if periodic[d]:
            a = np.pad(a, pw, mode="wrap")
        elif bc:
            a = np.pad(a, pw, mode="symmetric")
            sl_lo = [slice(None)] * 3
            sl_hi = [slice(None)] * 3
            sl_lo[d] = slice(0, ng)
            sl_hi[d] = slice(a.shape[d] - ng, a.shape[d])
            a[tuple(sl_lo)] *= -1.0
            a[tuple(sl_hi)] *= -1.0
        else:
            a = np.pad(a, pw, mode="constant", constant_values=np.nan)
    return a


def check(orc, dom_lo, dom_hi, periodic, boxes, ng, bc, seed=0, ncomp=1):
    shape = tuple(dom_hi[d] - dom_lo[d] + 1 for d in range(3))
    comps = [W.dyadic_codes(shape, seed + c) for c in range(ncomp)]
    # packed multi-component: per box, components slowest
    per_comp = [orc.pack(g, dom_lo, boxes, ng) for g in comps]
    packed = []
    offs = [0] * ncomp
    for lo, hi in boxes:
        n = int(np.prod(orc.box_shape(lo, hi, ng)))
        for c in range(ncomp):
            packed.append(per_comp[c][offs[c]:offs[c] + n])
            offs[c] += n
    packed = np.ascontiguousarray(np.concatenate(packed))
    orc.fill_boundary(dom_lo, dom_hi, periodic, boxes, ng, packed, ncomp=ncomp)
    if bc:
        orc.apply_bc(dom_lo, dom_hi, periodic, boxes, ng, packed, ncomp=ncomp)
    views = orc.box_views(packed, boxes, ng, ncomp)
    for c in range(ncomp):
        exp = padded_expect(comps[c], periodic, ng, bc)
        for (lo, hi), v in zip(boxes, views):
            vv = v[..., c] if ncomp > 1 else v
            s = tuple(slice(lo[d] - dom_lo[d], hi[d] - dom_lo[d] + 1 + 2 * ng) for d in range(3))
            e = exp[s]
            assert np.array_equal(vv, e, equal_nan=True), (lo, hi, c)


@pytest.mark.parametrize("periodic", [(1, 1, 1), (0, 0, 0), (1, 0, 1), (0, 1, 0)])
@pytest.mark.parametrize("bc", [False, True])
def test_fill_multibox(orc, periodic, bc):
    boxes = orc.chop((0, 0, 0), (15, 11, 7), 4)
    check(orc, (0, 0, 0), (15, 11, 7), periodic, boxes, 1, bc)


@pytest.mark.parametrize("bc", [False, True])
def test_fill_negative_lo_uneven_boxes(orc, bc):
    dlo, dhi = (-6, -4, -2), (7, 5, 9)
    boxes = orc.chop(dlo, dhi, 4)
    assert len({(hi[0] - lo[0]) for lo, hi in boxes}) > 1  # uneven widths
    check(orc, dlo, dhi, (1, 0, 1), boxes, 1, bc, seed=3)


@pytest.mark.parametrize("ng", [1, 2])
def test_fill_single_box_periodic_self_images(orc, ng):
    check(orc, (0, 0, 0), (5, 5, 5), (1, 1, 1), [((0, 0, 0), (5, 5, 5))], ng, False, seed=5)
    check(orc, (0, 0, 0), (5, 5, 5), (1, 1, 1), [((0, 0, 0), (5, 5, 5))], ng, True, seed=5)


def test_fill_two_cell_domain(orc):
    boxes = [((0, 0, 0), (0, 1, 1)), ((1, 0, 0), (1, 1, 1))]
    for per in [(1, 1, 1), (0, 0, 0), (1, 0, 0)]:
        check(orc, (0, 0, 0), (1, 1, 1), per, boxes, 1, False, seed=7)
        check(orc, (0, 0, 0), (1, 1, 1), per, boxes, 1, True, seed=7)


def test_fill_ng2_multibox_multicomp(orc):
    boxes = orc.chop((0, 0, 0), (11, 11, 7), 4)
    check(orc, (0, 0, 0), (11, 11, 7), (1, 0, 1), boxes, 2, False, seed=11, ncomp=2)
    check(orc, (0, 0, 0), (11, 11, 7), (1, 0, 1), boxes, 2, True, seed=11, ncomp=2)


def test_fill_leaves_uncovered_ghosts(orc):
    # a BoxArray that does not cover the domain: ghosts over the hole stay NaN
    dlo, dhi = (0, 0, 0), (7, 7, 7)
    boxes = [((0, 0, 0), (3, 7, 7)), ((6, 0, 0), (7, 7, 7))]
    glob = W.dyadic_codes((8, 8, 8), 1)
    packed = orc.pack(glob, dlo, boxes, 1)
    orc.fill_boundary(dlo, dhi, (1, 1, 1), boxes, 1, packed)
    v0, v1 = orc.box_views(packed, boxes, 1)
    assert np.isnan(v0[-1, 1:-1, 1:-1]).all()        # x = 4 lies in the hole
    assert np.array_equal(v0[0, 1:-1, 1:-1], glob[7])  # x = -1 wraps into box 1
    assert np.isnan(v1[0, 1:-1, 1:-1]).all()         # x = 5 lies in the hole
    # valid cells are never written
    assert np.array_equal(v0[1:-1, 1:-1, 1:-1], glob[0:4])


def test_fill_float32(orc):
    boxes = orc.chop((0, 0, 0), (7, 7, 7), 4)
    glob = W.dyadic_codes((8, 8, 8), 2)
    packed = orc.pack(glob, (0, 0, 0), boxes, 1, dtype=np.float32)
    orc.fill_boundary((0, 0, 0), (7, 7, 7), (1, 1, 1), boxes, 1, packed)
    exp = padded_expect(glob, (1, 1, 1), 1, False).astype(np.float32)
    for (lo, hi), v in zip(boxes, orc.box_views(packed, boxes, 1)):
        s = tuple(slice(lo[d], hi[d] + 3) for d in range(3))
        assert np.array_equal(v, exp[s])


@pytest.mark.parametrize("ng,ncomp,periodic", [(2, 2, (1, 0, 1)), (2, 1, (1, 1, 1)), (1, 3, (0, 1, 1))])
def test_fill_float32_multighost_multicomp(orc, ng, ncomp, periodic):
    # the FP32 exchange against numpy.pad, several ghost layers and components
    dlo, dhi = (0, 0, 0), (11, 11, 7)
    shape = (12, 12, 8)
    boxes = orc.chop(dlo, dhi, 4)
    comps = [W.dyadic_codes(shape, 20 + c) for c in range(ncomp)]
    per_comp = [orc.pack(g, dlo, boxes, ng, dtype=np.float32) for g in comps]
    packed, offs = [], [0] * ncomp
    for lo, hi in boxes:
        n = int(np.prod(orc.box_shape(lo, hi, ng)))
        for c in range(ncomp):
            packed.append(per_comp[c][offs[c]:offs[c] + n])
            offs[c] += n
    packed = np.ascontiguousarray(np.concatenate(packed))
    orc.fill_boundary(dlo, dhi, periodic, boxes, ng, packed, ncomp=ncomp)
    views = orc.box_views(packed, boxes, ng, ncomp)
    for c in range(ncomp):
        exp = padded_expect(comps[c], periodic, ng, False).astype(np.float32)
        for (lo, hi), v in zip(boxes, views):
            vv = v[..., c] if ncomp > 1 else v
            s = tuple(slice(lo[d] - dlo[d], hi[d] - dlo[d] + 1 + 2 * ng) for d in range(3))
            assert np.array_equal(vv, exp[s], equal_nan=True), (lo, hi, c)
