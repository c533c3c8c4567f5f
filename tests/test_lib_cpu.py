"""Host-side checks of the HIP library that need no GPU: the shared library
loads and exports every entry point the public header declares, and its
host logic (box chopping, the level hierarchy, MultiFab sizing, argument
validation, the Box API of the paper's Listing 9) agrees with the oracle and
the paper's worked example."""
import json
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")


@pytest.fixture(scope="module")
def bx():
    import paper_2403_12179_amd as bx
    return bx


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(bxmg_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol(bx):
    lib = bx.lib()
    names = declared_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.bxmg_version() >= 100


def test_library_has_gfx950_code():
    so = os.path.join(ROOT, "paper_2403_12179_amd", "libbxmg.so")
    assert b"amdgcn-amd-amdhsa--gfx950" in open(so, "rb").read()


def test_missing_library_fails_loudly(tmp_path):
    code = ("import paper_2403_12179_amd._lib as L; L.LIB_PATH = %r\n"
            "try:\n    L.lib()\nexcept ImportError as e:\n    print('IMPORTERROR', e)\n") % str(tmp_path / "nope.so")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT)
    assert "IMPORTERROR" in out.stdout


def test_box_listing9_worked_example(bx):
    g = json.load(open(os.path.join(GOLD, "box_listing9.json")))
    b = bx.Box(small=tuple(g["small"]), big=tuple(g["big"]))
    assert b.size == tuple(g["size"])
    assert b.ok is g["ok"]
    s = b.make_slab(g["make_slab"]["direction"], g["make_slab"]["slab_index"])
    assert s.size == tuple(g["make_slab"]["size"])
    assert repr(b) == "<Box of size '(3,4,5)'>"


@pytest.mark.parametrize("dom", [((0, 0, 0), (255, 255, 255)), ((0, 0, 0), (47, 95, 239)), ((-16, -8, 0), (15, 23, 39)),
                                 ((3, 5, 7), (40, 20, 12))])
@pytest.mark.parametrize("mb", [32, 16, 7])
def test_chop_matches_oracle(bx, orc, dom, mb):
    ba = bx.BoxArray.chop(dom[0], dom[1], mb)
    mine = [(b.small, b.big) for b in ba.boxes]
    assert mine == orc.chop(dom[0], dom[1], mb)


LIB_MIN_BOX_EDGE = 32  # the library's box-merging threshold (bxmg_boxarray_hierarchy)


@pytest.mark.parametrize("n,mb", [(256, 32), (512, 64), (48, 32), (96, 32), (240, 32), (64, 16), (32, 32), (6, 4)])
def test_hierarchy_matches_oracle(bx, orc, n, mb):
    # the library merges boxes once an edge drops below 32 (the oracle's
    # threshold is a parameter; the level domains do not depend on it)
    ba = bx.BoxArray.chop((0, 0, 0), (n - 1,) * 3, mb)
    boxes = [(b.small, b.big) for b in ba.boxes]
    mine = [(d.small, d.big, [(b.small, b.big) for b in bl]) for d, bl in ba.hierarchy()]
    assert mine == orc.hierarchy((0, 0, 0), (n - 1,) * 3, boxes, min_box_edge=LIB_MIN_BOX_EDGE)
    assert [(d[0], d[1]) for d in mine] == [(d[0], d[1]) for d in orc.hierarchy((0, 0, 0), (n - 1,) * 3, boxes)]


def test_boxarray_list_validation(bx):
    with pytest.raises(bx.BxmgError, match="overlap"):
        bx.BoxArray.from_boxes((0, 0, 0), (7, 7, 7), [((0, 0, 0), (4, 7, 7)), ((4, 0, 0), (7, 7, 7))])
    with pytest.raises(bx.BxmgError, match="leaves the domain"):
        bx.BoxArray.from_boxes((0, 0, 0), (7, 7, 7), [((0, 0, 0), (8, 7, 7))])
    with pytest.raises(bx.BxmgError, match="empty"):
        bx.BoxArray.from_boxes((0, 0, 0), (7, 7, 7), [((3, 0, 0), (2, 7, 7))])
    with pytest.raises(bx.BxmgError):
        bx.BoxArray.chop((0, 0, 0), (7, 7, 7), 0)
    ba = bx.BoxArray.from_boxes((0, 0, 0), (7, 7, 7), [((0, 0, 0), (3, 7, 7)), ((6, 0, 0), (7, 7, 7))])
    assert len(ba) == 2  # holes are allowed for FillBoundary


def test_multifab_bytes(bx):
    lib = bx.lib()
    ba = bx.BoxArray.chop((0, 0, 0), (255, 255, 255), 32)
    per_box = 34 ** 3 * 8
    per_box = (per_box + 255) // 256 * 256
    assert lib.bxmg_multifab_bytes(ba._h, 1, 1, 0) == 512 * per_box
    assert lib.bxmg_multifab_bytes(ba._h, 2, 2, 1) == 512 * ((36 ** 3 * 2 * 4 + 255) // 256 * 256)
    assert lib.bxmg_multifab_bytes(ba._h, 0, 1, 0) == 0


def test_workloads_are_deterministic():
    import workloads as W
    a = W.uniform_rhs((8, 8, 8), 2)
    b = W.uniform_rhs((8, 8, 8), 2)
    assert np.array_equal(a, b) and a.flags.f_contiguous
    beta = W.smooth_gaussian_beta((16, 16, 16), 33)
    g = np.log(beta)
    assert abs(g.mean()) < 1e-12 and abs(g.std() - 1.0) < 1e-12
    edges = W.batch_edges(256, 4)
    assert set(edges) <= {32, 48, 64, 96, 128} and len(edges) == 256
    tr = W.serving_trace(100, 5)
    assert all(32 <= r["edge"] <= 256 and r["edge"] % 16 == 0 for r in tr)
    assert all(1e-10 <= r["tol"] <= 1e-8 for r in tr)


@pytest.mark.parametrize("boxes", [[((0, 0, 0), (2, 7, 7)), ((3, 0, 0), (7, 7, 7))],
                                   [((0, 0, 0), (1, 7, 7)), ((2, 0, 0), (7, 7, 7))],
                                   [((-4, 0, 0), (-1, 7, 7)), ((0, 0, 0), (3, 7, 7))]])
def test_hierarchy_of_box_lists_matches_oracle(bx, orc, boxes):
    dlo = (min(b[0][0] for b in boxes), 0, 0)
    dhi = (max(b[1][0] for b in boxes), 7, 7)
    ba = bx.BoxArray.from_boxes(dlo, dhi, boxes)
    mine = [(d.small, d.big, [(b.small, b.big) for b in bl]) for d, bl in ba.hierarchy()]
    assert mine == orc.hierarchy(dlo, dhi, boxes, min_box_edge=LIB_MIN_BOX_EDGE)
