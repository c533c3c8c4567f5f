"""ctypes wrapper around the C++ oracle (``mg_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the oracle is the plain, single-threaded FP64
reference for the multigrid path.  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import this module; the product library
never does.  It shares no code with the HIP library.

Global arrays are numpy arrays of shape (nx, ny, nz) over the domain, Fortran
order (x fastest), matching the FArrayBox order of the paper (Section 2 and
Section 4.1, "Fortran order").  Multi-box arrays are "packed": the grown boxes
of a level one after another, each F-order, component slowest.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

CFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (no FMA contraction, no -march=native)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", *CFLAGS, "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("nu1", C.c_int), ("nu2", C.c_int), ("max_cycles", C.c_int), ("precision", C.c_int),
                ("prolong", C.c_int), ("fixed_cycles", C.c_int), ("rel_tol", C.c_double),
                ("abs_tol", C.c_double), ("h", C.c_double), ("bottom_rtol", C.c_double),
                ("min_box_edge", C.c_int), ("krylov", C.c_int), ("use_guess", C.c_int), ("pad", C.c_int),
                ("alpha", C.c_double)]


class Info(C.Structure):
    _fields_ = [("status", C.c_int), ("cycles", C.c_int), ("nhist", C.c_int), ("levels", C.c_int),
                ("rel_inf", C.c_double), ("rel_l2", C.c_double), ("f_inf", C.c_double),
                ("hist", C.c_double * 256), ("hist_l2", C.c_double * 256), ("cg_iters_max", C.c_int)]


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = C.CDLL(_LIB)
        _lib.orc_faces.restype = C.c_long
    return _lib


# ----------------------------------------------------------------- helpers
def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _i32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32).ravel())


def dom6(lo, hi):
    return _i32(list(lo) + list(hi))


def lohi_array(boxes):
    """boxes: list of (lo, hi) triples -> int32 [nb*6]."""
    return _i32([list(lo) + list(hi) for lo, hi in boxes]) if boxes else np.zeros(0, np.int32)


def box_shape(lo, hi, ng=0):
    return tuple(hi[d] - lo[d] + 1 + 2 * ng for d in range(3))


def packed_size(boxes, ng, ncomp=1):
    return sum(int(np.prod(box_shape(lo, hi, ng))) for lo, hi in boxes) * ncomp


def pack(glob, dom_lo, boxes, ng, ghost=np.nan, dtype=np.float64):
    """Scatter a global F-order array into packed grown boxes; ghosts = ghost."""
    out = []
    for lo, hi in boxes:
        a = np.full(box_shape(lo, hi, ng), ghost, dtype=dtype, order="F")
        s = tuple(slice(lo[d] - dom_lo[d], hi[d] - dom_lo[d] + 1) for d in range(3))
        a[ng:a.shape[0] - ng, ng:a.shape[1] - ng, ng:a.shape[2] - ng] = glob[s]
        out.append(a.ravel(order="F"))
    return np.ascontiguousarray(np.concatenate(out)) if out else np.zeros(0, dtype)


def box_views(packed, boxes, ng, ncomp=1):
    """Per-box F-order views (shape grown box [, ncomp]) into a packed array."""
    views, off = [], 0
    for lo, hi in boxes:
        sh = box_shape(lo, hi, ng)
        n = int(np.prod(sh))
        v = packed[off:off + n * ncomp]
        views.append(v.reshape(sh + ((ncomp,) if ncomp > 1 else ()), order="F"))
        off += n * ncomp
    return views


def unpack_valid(packed, dom_lo, dom_hi, boxes, ng, dtype=np.float64):
    glob = np.full(box_shape(dom_lo, dom_hi), np.nan, dtype=dtype, order="F")
    for (lo, hi), v in zip(boxes, box_views(packed, boxes, ng)):
        s = tuple(slice(lo[d] - dom_lo[d], hi[d] - dom_lo[d] + 1) for d in range(3))
        glob[s] = v[ng:v.shape[0] - ng, ng:v.shape[1] - ng, ng:v.shape[2] - ng]
    return glob


# -------------------------------------------------------------- box arrays
def chop(dom_lo, dom_hi, max_box):
    L = lib()
    cap = 1 << 20
    out = np.zeros(cap * 6, np.int32)
    n = L.orc_chop(_ip(dom6(dom_lo, dom_hi)), int(max_box), cap, _ip(out))
    assert n >= 0
    return [(tuple(int(x) for x in out[6 * b:6 * b + 3]), tuple(int(x) for x in out[6 * b + 3:6 * b + 6])) for b in range(n)]


def hierarchy(dom_lo, dom_hi, boxes, min_box_edge=0):
    """List of (dom_lo, dom_hi, boxes) per multigrid level.  Boxes coarsen one
    by one while every box edge is >= min_box_edge (0: the oracle's default,
    4), else the coarse level is one box."""
    L = lib()
    capl, capb = 64, 1 << 20
    nb = np.zeros(capl, np.int32)
    d6 = np.zeros(capl * 6, np.int32)
    lh = np.zeros(capb * 6, np.int32)
    nl = L.orc_hierarchy(_ip(dom6(dom_lo, dom_hi)), len(boxes), _ip(lohi_array(boxes)), int(min_box_edge), capl,
                         capb, _ip(nb), _ip(d6), _ip(lh))
    assert nl > 0
    levels, o = [], 0
    for l in range(nl):
        bl = []
        for _ in range(nb[l]):
            bl.append((tuple(int(x) for x in lh[6 * o:6 * o + 3]), tuple(int(x) for x in lh[6 * o + 3:6 * o + 6])))
            o += 1
        levels.append((tuple(int(x) for x in d6[6 * l:6 * l + 3]), tuple(int(x) for x in d6[6 * l + 3:6 * l + 6]), bl))
    return levels


# ------------------------------------------------------------ level stages
def fill_boundary(dom_lo, dom_hi, periodic, boxes, ng, packed, ncomp=1):
    """FillBoundary in place on a packed FP64 (or FP32) multi-box array."""
    L = lib()
    assert packed.flags.c_contiguous and packed.size == packed_size(boxes, ng, ncomp)
    if packed.dtype == np.float32:
        L.orc_fill_boundary_f32(_ip(dom6(dom_lo, dom_hi)), _ip(_i32(periodic)), len(boxes), _ip(lohi_array(boxes)),
                                int(ng), int(ncomp), _fp(packed))
        return packed
    assert packed.dtype == np.float64
    L.orc_fill_boundary(_ip(dom6(dom_lo, dom_hi)), _ip(_i32(periodic)), len(boxes), _ip(lohi_array(boxes)), int(ng),
                        int(ncomp), _dp(packed))
    return packed


def apply_bc(dom_lo, dom_hi, periodic, boxes, ng, packed, ncomp=1, odd=True):
    L = lib()
    assert packed.dtype == np.float64 and packed.size == packed_size(boxes, ng, ncomp)
    L.orc_apply_bc(_ip(dom6(dom_lo, dom_hi)), _ip(_i32(periodic)), len(boxes), _ip(lohi_array(boxes)), int(ng),
                   int(ncomp), int(bool(odd)), _dp(packed))
    return packed


def gs(dom_lo, dom_hi, periodic, boxes, h, colour, u, f, beta_glob=None, alpha=0.0):
    """One red-black colour (ng = 1, ghosts of u current) in place on u."""
    L = lib()
    if u.dtype == np.float32:
        assert beta_glob is None and alpha == 0.0
        L.orc_gs_f32(_ip(dom6(dom_lo, dom_hi)), _ip(_i32(periodic)), len(boxes), _ip(lohi_array(boxes)),
                     C.c_double(h), int(colour), _fp(u), _fp(f))
        return u
    b = None if beta_glob is None else np.asfortranarray(beta_glob, dtype=np.float64)
    L.orc_gs(_ip(dom6(dom_lo, dom_hi)), _ip(_i32(periodic)), len(boxes), _ip(lohi_array(boxes)), C.c_double(h),
             int(colour), _dp(u), _dp(f), _dp(b.ravel(order="F")) if b is not None else None, C.c_double(alpha))
    return u


def residual(dom_lo, dom_hi, periodic, boxes, h, u, f, beta_glob=None, alpha=0.0):
    """r = f - L u on valid cells (packed, ng = 1); returns (r, rinf, rl2sq)."""
    L = lib()
    r = np.zeros_like(u)
    norms = np.zeros(2)
    b = None if beta_glob is None else np.asfortranarray(beta_glob, dtype=np.float64).ravel(order="F")
    L.orc_residual(_ip(dom6(dom_lo, dom_hi)), _ip(_i32(periodic)), len(boxes), _ip(lohi_array(boxes)),
                   C.c_double(h), _dp(u), _dp(f), _dp(b), C.c_double(alpha), _dp(r), _dp(norms))
    return r, norms[0], norms[1]


def restrict(fine_boxes, ngf, coarse_boxes, ngc, rf, fc=None):
    L = lib()
    if fc is None:
        fc = np.zeros(packed_size(coarse_boxes, ngc))
    L.orc_restrict(len(fine_boxes), _ip(lohi_array(fine_boxes)), int(ngf), len(coarse_boxes),
                   _ip(lohi_array(coarse_boxes)), int(ngc), _dp(rf), _dp(fc))
    return fc


def prolong(fine_boxes, ngf, coarse_boxes, ngc, ec, uf, order=2):
    L = lib()
    L.orc_prolong(len(fine_boxes), _ip(lohi_array(fine_boxes)), int(ngf), len(coarse_boxes),
                  _ip(lohi_array(coarse_boxes)), int(ngc), int(order), _dp(ec), _dp(uf))
    return uf


def faces(dom_lo, dom_hi, periodic, boxes, beta_glob):
    """Per level: (bx, by, bz) global face arrays (F-order, face index first)."""
    L = lib()
    levels = hierarchy(dom_lo, dom_hi, boxes)
    n = 0
    shapes = []
    for dlo, dhi, _ in levels:
        sh = box_shape(dlo, dhi)
        s3 = [tuple(sh[e] + (e == d) for e in range(3)) for d in range(3)]
        shapes.append(s3)
        n += sum(int(np.prod(s)) for s in s3)
    out = np.zeros(n)
    b = np.asfortranarray(beta_glob, dtype=np.float64).ravel(order="F")
    got = L.orc_faces(_ip(dom6(dom_lo, dom_hi)), _ip(_i32(periodic)), len(boxes), _ip(lohi_array(boxes)), _dp(b),
                      _dp(out), C.c_long(n))
    assert got == n
    res, o = [], 0
    for s3 in shapes:
        lv = []
        for s in s3:
            m = int(np.prod(s))
            lv.append(out[o:o + m].reshape(s, order="F"))
            o += m
        res.append(tuple(lv))
    return res


def apply_op(dom_lo, dom_hi, periodic, h, u_glob, beta_glob=None, alpha=0.0):
    """L u = div(beta grad u) - alpha u on a global array (FP64)."""
    L = lib()
    u = np.asfortranarray(u_glob, dtype=np.float64)
    out = np.zeros(u.shape, order="F")
    b = None if beta_glob is None else np.asfortranarray(beta_glob, dtype=np.float64)
    L.orc_apply_op(_ip(dom6(dom_lo, dom_hi)), _ip(_i32(periodic)), C.c_double(h), _dp(u.ravel(order="F")),
                   _dp(b.ravel(order="F")) if b is not None else None, C.c_double(alpha),
                   _dp(out.ravel(order="F")))
    return out


def bottom(dom_lo, dom_hi, periodic, h, f_glob, beta_glob=None, rtol=1e-12, alpha=0.0):
    L = lib()
    f = np.asfortranarray(f_glob, dtype=np.float64)
    u = np.zeros(f.shape, order="F")
    b = None if beta_glob is None else np.asfortranarray(beta_glob, dtype=np.float64)
    it = C.c_int(0)
    L.orc_bottom(_ip(dom6(dom_lo, dom_hi)), _ip(_i32(periodic)), C.c_double(h), _dp(f.ravel(order="F")),
                 _dp(b.ravel(order="F")) if b is not None else None, C.c_double(alpha), C.c_double(rtol),
                 _dp(u.ravel(order="F")),
                 C.byref(it))
    return u, it.value


def solve(dom_lo, dom_hi, periodic, boxes, f_glob, beta_glob=None, h=None, nu1=2, nu2=2, max_cycles=200,
          precision=0, prolong=2, fixed_cycles=0, rel_tol=1e-10, abs_tol=0.0, bottom_rtol=1e-12, min_box_edge=0,
          krylov=0, alpha=0.0, u0=None):
    """Full multigrid solve of div(beta grad u) - alpha u = f; returns
    (u_glob, info dict).  min_box_edge: the hierarchy's box-merging threshold
    (0: default).  krylov=1: conjugate gradients preconditioned by one
    V-cycle per iteration (cycles counts the iterations).  u0: initial guess
    (default zero)."""
    L = lib()
    f = np.asfortranarray(f_glob, dtype=np.float64)
    assert f.shape == box_shape(dom_lo, dom_hi)
    if h is None:
        h = 1.0 / f.shape[0]
    p = Params(nu1, nu2, max_cycles, precision, prolong, fixed_cycles, rel_tol, abs_tol, h, bottom_rtol,
               int(min_box_edge), int(krylov), int(u0 is not None), 0, float(alpha))
    info = Info()
    u = np.zeros(f.shape, order="F") if u0 is None else np.array(u0, dtype=np.float64, order="F", copy=True)
    b = None if beta_glob is None else np.asfortranarray(beta_glob, dtype=np.float64)
    L.orc_solve(C.byref(p), _ip(dom6(dom_lo, dom_hi)), _ip(_i32(periodic)), len(boxes), _ip(lohi_array(boxes)),
                _dp(f.ravel(order="F")), _dp(b.ravel(order="F")) if b is not None else None,
                _dp(u.ravel(order="F")), C.byref(info))
    return u, _info_dict(info)


def _info_dict(info):
    return {"status": info.status, "cycles": info.cycles, "levels": info.levels, "rel_inf": info.rel_inf,
            "rel_l2": info.rel_l2, "f_inf": info.f_inf, "hist": list(info.hist[:info.nhist]),
            "hist_l2": list(info.hist_l2[:info.nhist]), "cg_iters_max": info.cg_iters_max}


def heat_step(dom_lo, dom_hi, periodic, boxes, u_glob, dt, source=None, beta_glob=None, h=None, **kw):
    """One backward-Euler step of u_t = div(beta grad u) + source: the
    Helmholtz solve with alpha = 1/dt and f = -(u/dt + source), started from
    u.  Returns (u', info dict); kw as for solve (nu1, precision, krylov ...)."""
    L = lib()
    u = np.array(u_glob, dtype=np.float64, order="F", copy=True)
    assert u.shape == box_shape(dom_lo, dom_hi)
    if h is None:
        h = 1.0 / u.shape[0]
    names = ("nu1", "nu2", "max_cycles", "precision", "prolong", "fixed_cycles", "rel_tol", "abs_tol",
             "bottom_rtol", "min_box_edge", "krylov")
    defaults = dict(nu1=2, nu2=2, max_cycles=200, precision=0, prolong=2, fixed_cycles=0, rel_tol=1e-10,
                    abs_tol=0.0, bottom_rtol=1e-12, min_box_edge=0, krylov=0)
    defaults.update(kw)
    v = [defaults[n] for n in names]
    p = Params(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], h, v[8], int(v[9]), int(v[10]), 1, 0, 0.0)
    info = Info()
    s = None if source is None else np.asfortranarray(source, dtype=np.float64)
    b = None if beta_glob is None else np.asfortranarray(beta_glob, dtype=np.float64)
    L.orc_heat_step(C.byref(p), _ip(dom6(dom_lo, dom_hi)), _ip(_i32(periodic)), len(boxes), _ip(lohi_array(boxes)),
                    C.c_double(dt), _dp(s.ravel(order="F")) if s is not None else None,
                    _dp(b.ravel(order="F")) if b is not None else None, _dp(u.ravel(order="F")), C.byref(info))
    return u, _info_dict(info)


# ------------------------------------------------------------------- nodal
# Node arrays: (n0+1, n1+1, n2+1) values over the domain's nodes, F-order.

def _nodal_args(n, periodic):
    return _ip(_i32(n)), _ip(_i32(periodic))


def nodal_shape(n):
    return tuple(int(x) + 1 for x in n)


def nodal_solve(n, periodic, f, h=None, nu1=2, nu2=2, max_cycles=200, fixed_cycles=0, rel_tol=1e-10,
                bottom_rtol=1e-12):
    """Nodal Poisson solve (FP64 V-cycles); returns (u, info dict)."""
    L = lib()
    f = np.asfortranarray(f, dtype=np.float64)
    assert f.shape == nodal_shape(n)
    h = 1.0 / n[0] if h is None else h
    u = np.zeros(f.shape, order="F")
    info = Info()
    L.orc_nodal_solve(*_nodal_args(n, periodic), C.c_double(h), int(nu1), int(nu2), int(max_cycles),
                      int(fixed_cycles), C.c_double(rel_tol), C.c_double(bottom_rtol), _dp(f.ravel(order="F")),
                      _dp(u.ravel(order="F")), C.byref(info))
    return u, _info_dict(info)


def nodal_apply(n, periodic, h, u):
    L = lib()
    u = np.asfortranarray(u, dtype=np.float64)
    out = np.zeros(u.shape, order="F")
    L.orc_nodal_apply(*_nodal_args(n, periodic), C.c_double(h), _dp(u.ravel(order="F")), _dp(out.ravel(order="F")))
    return out


def nodal_gs(n, periodic, h, colour, u, f):
    L = lib()
    u = np.array(u, dtype=np.float64, order="F", copy=True)
    f = np.asfortranarray(f, dtype=np.float64)
    L.orc_nodal_gs(*_nodal_args(n, periodic), C.c_double(h), int(colour), _dp(u.ravel(order="F")),
                   _dp(f.ravel(order="F")))
    return u


def nodal_residual(n, periodic, h, u, f):
    L = lib()
    u = np.asfortranarray(u, dtype=np.float64)
    f = np.asfortranarray(f, dtype=np.float64)
    r = np.zeros(u.shape, order="F")
    norms = np.zeros(2)
    L.orc_nodal_residual(*_nodal_args(n, periodic), C.c_double(h), _dp(u.ravel(order="F")), _dp(f.ravel(order="F")),
                         _dp(r.ravel(order="F")), _dp(norms))
    return r, norms[0], norms[1]


def nodal_restrict(n, periodic, rf):
    L = lib()
    rf = np.asfortranarray(rf, dtype=np.float64)
    fc = np.zeros(nodal_shape([x // 2 for x in n]), order="F")
    L.orc_nodal_restrict(*_nodal_args(n, periodic), _dp(rf.ravel(order="F")), _dp(fc.ravel(order="F")))
    return fc


def nodal_prolong_add(n, periodic, ec, uf):
    """uf (fine grid of n cells) += P ec (coarse grid of n/2 cells)."""
    L = lib()
    ec = np.asfortranarray(ec, dtype=np.float64)
    uf = np.array(uf, dtype=np.float64, order="F", copy=True)
    L.orc_nodal_prolong_add(*_nodal_args(n, periodic), _dp(ec.ravel(order="F")), _dp(uf.ravel(order="F")))
    return uf


def nodal_bottom(n, periodic, h, f, rtol=1e-12):
    L = lib()
    f = np.asfortranarray(f, dtype=np.float64)
    u = np.zeros(f.shape, order="F")
    it = L.orc_nodal_bottom(*_nodal_args(n, periodic), C.c_double(h), _dp(f.ravel(order="F")),
                            _dp(u.ravel(order="F")), C.c_double(rtol))
    return u, it


def parallel_copy(dom_lo, dom_hi, periodic, dst_boxes, dst_ng, dst, src_boxes, src_ng, src, ncomp=1,
                  dst_ncomp=1, src_ncomp=1, dcomp=0, scomp=0, copy_ng=0):
    """ParallelCopy from a packed source (src_boxes, src_ng, src_ncomp
    components) into a copy of a packed destination; returns the result."""
    L = lib()
    out = np.array(dst, dtype=np.float64, copy=True)
    src = np.ascontiguousarray(src, dtype=np.float64)
    assert out.size == packed_size(dst_boxes, dst_ng, dst_ncomp) and src.size == packed_size(src_boxes, src_ng, src_ncomp)
    L.orc_parallel_copy(_ip(dom6(dom_lo, dom_hi)), _ip(_i32(periodic)), len(dst_boxes), _ip(lohi_array(dst_boxes)),
                        int(dst_ng), int(dst_ncomp), int(copy_ng), len(src_boxes), _ip(lohi_array(src_boxes)),
                        int(src_ng), int(src_ncomp), int(dcomp), int(scomp), int(ncomp), _dp(out), _dp(src))
    return out


# ------------------------------------------------------------ composite
def composite_solve(n, periodic, coarse_boxes, fine_boxes, fc, ff, h=None, nu1=2, nu2=2, max_cycles=100,
                    fixed_cycles=0, rel_tol=1e-10):
    """Two-level composite solve: coarse level over [0, n)^3 (coarse_boxes),
    fine level (ratio 2) over fine_boxes in fine indices.  fc: coarse rhs
    (n^3, read at uncovered cells), ff: fine rhs over the refined domain
    ((2n)^3, read inside fine boxes).  Returns (uc, uf, info)."""
    L = lib()
    n = int(n)
    h = 1.0 / n if h is None else h
    fc = np.asfortranarray(fc, dtype=np.float64)
    ff = np.asfortranarray(ff, dtype=np.float64)
    assert fc.shape == (n, n, n) and ff.shape == (2 * n, 2 * n, 2 * n)
    uc = np.zeros((n, n, n), order="F")
    uf = np.zeros((2 * n, 2 * n, 2 * n), order="F")
    info = Info()
    L.orc_composite_solve(_ip(dom6((0, 0, 0), (n - 1,) * 3)), _ip(_i32(periodic)), len(coarse_boxes),
                          _ip(lohi_array(coarse_boxes)), len(fine_boxes), _ip(lohi_array(fine_boxes)), C.c_double(h),
                          int(nu1), int(nu2), int(max_cycles), int(fixed_cycles), C.c_double(rel_tol),
                          _dp(fc.ravel(order="F")), _dp(ff.ravel(order="F")), _dp(uc.ravel(order="F")),
                          _dp(uf.ravel(order="F")), C.byref(info))
    return uc, uf, _info_dict(info)


def composite_apply(n, periodic, coarse_boxes, fine_boxes, h, uc, uf):
    """The composite operator: (Lc, Lf) with Lc zero at covered coarse cells
    and Lf zero outside the fine boxes.  Covered coarse values are replaced
    by the mean of their children first."""
    L = lib()
    n = int(n)
    uc = np.asfortranarray(uc, dtype=np.float64)
    uf = np.asfortranarray(uf, dtype=np.float64)
    Lc = np.zeros((n, n, n), order="F")
    Lf = np.zeros((2 * n, 2 * n, 2 * n), order="F")
    st = L.orc_composite_apply(_ip(dom6((0, 0, 0), (n - 1,) * 3)), _ip(_i32(periodic)), len(coarse_boxes),
                               _ip(lohi_array(coarse_boxes)), len(fine_boxes), _ip(lohi_array(fine_boxes)),
                               C.c_double(h), _dp(uc.ravel(order="F")), _dp(uf.ravel(order="F")),
                               _dp(Lc.ravel(order="F")), _dp(Lf.ravel(order="F")))
    if st != 0:
        raise ValueError("composite layout not supported")
    return Lc, Lf
