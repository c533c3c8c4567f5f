"""The allocation-free ghost exchange, bxmg_fill_boundary_noalloc, against
bxmg_fill_boundary through the C ABI: the ghost cells it writes (and the
ones it must leave alone, NaN sentinels) are bitwise those of the
allocating call, on calls in a row on one stream -- a large MultiFab, then a
smaller one, then the large one again -- each of which overwrites the
shared staging array.  A region list beyond the array is refused on the
host before anything is launched."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bx():
    import paper_2403_12179_amd as bx
    return bx


def make(bx, dlo, dhi, mb, per, ng, ncomp, dtype, seed):
    bc = tuple(bx.PERIODIC if p else bx.DIRICHLET0 for p in per)
    ba = bx.BoxArray.chop(dlo, dhi, mb, bc=bc)
    shape = tuple(dhi[d] - dlo[d] + 1 for d in range(3))
    pair = []
    for _ in range(2):
        mf = bx.MultiFab(ba, ncomp=ncomp, nghost=ng, dtype=dtype).set_val(np.nan)
        for c in range(ncomp):
            mf.from_global(W.dyadic_codes(shape, seed + c), comp=c)
        pair.append(mf)
    return ba, pair


CASES = [  # large first, then smaller: (dom_lo, dom_hi, max_box, periodic, nghost, ncomp, dtype)
    ((0, 0, 0), (127, 127, 127), 16, (1, 1, 1), 2, 2, "f64"),  # 512 boxes, 26 regions each
    ((-6, -4, -2), (9, 7, 13), 4, (1, 0, 1), 1, 1, "f32"),
]


def test_noalloc_fill_equals_fill(bx):
    lib = bx.lib()
    sets = [make(bx, *c, seed=300 + 10 * q) for q, c in enumerate(CASES)]
    order = [0, 1, 0]
    for q in order:  # no synchronisation between the calls
        _, (a, b) = sets[q]
        s = C.c_void_p(a.ctx.stream.cuda_stream)
        for cross in (0,):
            bx._lib.check(lib.bxmg_fill_boundary(a._h, 0, a.ncomp, cross, s))
            bx._lib.check(lib.bxmg_fill_boundary_noalloc(b._h, 0, b.ncomp, cross, s))
    for q, (_, (a, b)) in enumerate(sets):
        pa, pb = a.to_packed(), b.to_packed()
        assert np.array_equal(pa, pb, equal_nan=True), q
        assert np.count_nonzero(np.isnan(pa)) < pa.size  # something was filled
    # one component, faces only, on the small MultiFab after the large one
    _, (a, b) = make(bx, *CASES[1], seed=400)
    s = C.c_void_p(a.ctx.stream.cuda_stream)
    bx._lib.check(lib.bxmg_fill_boundary_noalloc(sets[0][1][1]._h, 1, 1, 0, s))
    bx._lib.check(lib.bxmg_fill_boundary(a._h, 0, 1, 1, s))
    bx._lib.check(lib.bxmg_fill_boundary_noalloc(b._h, 0, 1, 1, s))
    assert np.array_equal(a.to_packed(), b.to_packed(), equal_nan=True)


def test_noalloc_fill_refuses_oversized_list(bx):
    # 4096 periodic boxes of 4^3: 26 regions each, beyond the staging array
    ba = bx.BoxArray.chop((0, 0, 0), (63, 63, 63), 4, bc=(bx.PERIODIC,) * 3)
    mf = bx.MultiFab(ba).set_val(1.0)
    st = bx.lib().bxmg_fill_boundary_noalloc(mf._h, 0, 1, 0, None)
    assert st == -1
    assert b"staging" in bx.lib().bxmg_last_error()
