"""Oracle pins: box chopping and the multigrid level hierarchy.

Chopping follows the reading in which a domain edge n is cut with blocking
factor bf = the largest power of two dividing n (capped at max_box_size) into
pieces of floor(max/bf)*bf plus one remainder; coarsening halves every box
while every box edge is even and >= 4 (lower corner even), otherwise the
coarse level is a single box; the domain halves while every edge is even and
>= 4.  The pins are worked examples and invariants that any mistake in the
index arithmetic (floor division of negative bounds, overlap, coverage) breaks.
"""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def edges_along(boxes, d):
    return sorted({(lo[d], hi[d]) for lo, hi in boxes})


@pytest.mark.parametrize("n,expect", [
    (48, [32, 16]), (96, [32, 32, 32]), (240, [32] * 7 + [16]), (208, [32] * 6 + [16]), (256, [32] * 8),
    (32, [32]), (16, [16]), (40, [32, 8]), (6, [6]), (33, [32, 1]),
])
def test_chop_worked_examples(orc, n, expect):
    boxes = orc.chop((0, 0, 0), (n - 1, 7, 7), 32)
    lens = [hi - lo + 1 for lo, hi in edges_along(boxes, 0)]
    assert lens == expect


def test_chop_geometry_of_fused_triad(orc):
    # Section 3.2: 512 patches of 32^3 make up the 256^3 domain.
    g = json.load(open(os.path.join(GOLD, "triad_fusion_geometry.json")))
    boxes = orc.chop(tuple(g["domain_lo"]), tuple(g["domain_hi"]), g["max_box_size"])
    assert len(boxes) == g["nboxes"]
    for lo, hi in boxes:
        assert [hi[d] - lo[d] + 1 for d in range(3)] == g["box_size"]


@pytest.mark.parametrize("dom_lo,dom_hi,mb", [((0, 0, 0), (47, 63, 95), 32), ((-16, -16, -16), (15, 15, 15), 16),
                                              ((-5, 3, 0), (10, 12, 20), 8)])
def test_chop_tiles_domain_exactly(orc, dom_lo, dom_hi, mb):
    boxes = orc.chop(dom_lo, dom_hi, mb)
    shape = tuple(dom_hi[d] - dom_lo[d] + 1 for d in range(3))
    cover = np.zeros(shape, np.int32)
    for lo, hi in boxes:
        assert all(hi[d] - lo[d] + 1 <= mb for d in range(3))
        cover[tuple(slice(lo[d] - dom_lo[d], hi[d] - dom_lo[d] + 1) for d in range(3))] += 1
    assert (cover == 1).all()


def test_hierarchy_single_box_32(orc):
    lv = orc.hierarchy((0, 0, 0), (31, 31, 31), [((0, 0, 0), (31, 31, 31))])
    assert [l[1][0] + 1 for l in lv] == [32, 16, 8, 4, 2]
    assert all(len(l[2]) == 1 for l in lv)


def test_hierarchy_256_in_512_boxes(orc):
    # boxes halve one by one while every box edge is even and >= 4
    # (32, 16, 8, 4, 2); 2-cell boxes cannot halve again, so the next level
    # is one box, which keeps halving down to the 2^3 bottom
    boxes = orc.chop((0, 0, 0), (255, 255, 255), 32)
    lv = orc.hierarchy((0, 0, 0), (255, 255, 255), boxes)
    assert [l[1][0] + 1 for l in lv] == [256, 128, 64, 32, 16, 8, 4, 2]
    assert [len(l[2]) for l in lv] == [512, 512, 512, 512, 512, 1, 1, 1]
    assert lv[4][2][0] == ((0, 0, 0), (1, 1, 1))
    # boxes coarsen one by one with floor division
    for (lo, hi), (clo, chi) in zip(lv[0][2], lv[1][2]):
        assert clo == tuple(x // 2 for x in lo) and chi == tuple(x // 2 for x in hi)


def test_hierarchy_negative_lower_corner(orc):
    boxes = orc.chop((-64, -64, -64), (63, 63, 63), 32)
    lv = orc.hierarchy((-64, -64, -64), (63, 63, 63), boxes)
    assert lv[1][0] == (-32, -32, -32) and lv[1][1] == (31, 31, 31)
    assert sorted(lv[1][2]) == sorted(((tuple(x // 2 for x in lo), tuple(x // 2 for x in hi)) for lo, hi in boxes))
    # floor division below zero: the box [-64, -33] halves to [-32, -17]
    assert ((-32, -32, -32), (-17, -17, -17)) in lv[1][2]
    assert [len(l[2]) for l in lv] == [64, 64, 64, 64, 64, 1, 1]
    assert lv[5][2] == [((-2, -2, -2), (1, 1, 1))]


@pytest.mark.parametrize("min_edge,counts", [(32, [512, 512, 1, 1, 1, 1, 1, 1]), (8, [512, 512, 512, 512, 1, 1, 1, 1]),
                                             (1 << 20, [512, 1, 1, 1, 1, 1, 1, 1])])
def test_hierarchy_merge_threshold(orc, min_edge, counts):
    # the threshold moves where boxes are merged, never the level domains
    boxes = orc.chop((0, 0, 0), (255, 255, 255), 32)
    lv = orc.hierarchy((0, 0, 0), (255, 255, 255), boxes, min_box_edge=min_edge)
    assert [l[1][0] + 1 for l in lv] == [256, 128, 64, 32, 16, 8, 4, 2]
    assert [len(l[2]) for l in lv] == counts


@pytest.mark.parametrize("n,bottom", [(48, 3), (96, 3), (64, 2), (80, 5), (112, 7), (240, 15)])
def test_hierarchy_odd_bottoms(orc, n, bottom):
    boxes = orc.chop((0, 0, 0), (n - 1, n - 1, n - 1), 32)
    lv = orc.hierarchy((0, 0, 0), (n - 1, n - 1, n - 1), boxes)
    assert lv[-1][1][0] + 1 == bottom
    assert len(lv[-1][2]) == 1
    # every level's boxes tile that level's domain
    for dlo, dhi, bl in lv:
        ncell = sum(int(np.prod([hi[d] - lo[d] + 1 for d in range(3)])) for lo, hi in bl)
        assert ncell == int(np.prod([dhi[d] - dlo[d] + 1 for d in range(3)]))


def test_hierarchy_stops_on_boxes_without_whole_pairs(orc):
    # a box with an odd lower corner cannot hand whole 2x2x2 blocks to a coarse
    # cell, so the level is the bottom even though the domain could halve
    boxes = [((0, 0, 0), (2, 7, 7)), ((3, 0, 0), (7, 7, 7))]
    lv = orc.hierarchy((0, 0, 0), (7, 7, 7), boxes)
    assert len(lv) == 1
    boxes = [((0, 0, 0), (1, 7, 7)), ((2, 0, 0), (7, 7, 7))]  # whole pairs, box of width 2
    lv = orc.hierarchy((0, 0, 0), (7, 7, 7), boxes)
    assert [l[1][0] + 1 for l in lv] == [8, 4, 2] and len(lv[1][2]) == 1
