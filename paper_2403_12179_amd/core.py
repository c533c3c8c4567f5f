"""Box, BoxArray, Context and MultiFab: thin Python objects over the C ABI.

Names and behaviour follow the paper's data model and Python bindings
(Section 2; Section 4, Listing 9 for Box; Section 4.1 for zero-copy views in
Fortran or C index order).  PyTorch provides device memory and streams only:
a MultiFab's slab is a caller-owned torch buffer handed to the library.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L


# ----------------------------------------------------------------------- Box
@dataclass(frozen=True)
class Box:
    """Inclusive integer index box (cell centred), global indices."""
    small: tuple
    big: tuple

    def __init__(self, small=(0, 0, 0), big=(0, 0, 0)):
        object.__setattr__(self, "small", tuple(int(x) for x in small))
        object.__setattr__(self, "big", tuple(int(x) for x in big))

    @property
    def size(self):
        return tuple(self.big[d] - self.small[d] + 1 for d in range(3))

    @property
    def ok(self):
        return all(self.big[d] >= self.small[d] for d in range(3))

    @property
    def numPts(self):
        s = self.size
        return s[0] * s[1] * s[2] if self.ok else 0

    def make_slab(self, direction, slab_index):
        """Flatten the box to the single index slab_index along direction."""
        lo, hi = list(self.small), list(self.big)
        lo[direction] = hi[direction] = int(slab_index)
        return Box(lo, hi)

    def grow(self, n):
        n = (n, n, n) if np.isscalar(n) else tuple(n)
        return Box([self.small[d] - n[d] for d in range(3)], [self.big[d] + n[d] for d in range(3)])

    def coarsen(self, r=2):
        return Box([self.small[d] // r for d in range(3)], [self.big[d] // r for d in range(3)])

    def __repr__(self):
        return "<Box of size '(%d,%d,%d)'>" % self.size


# ------------------------------------------------------------------ BoxArray
class BoxArray:
    """Disjoint boxes in a domain with a boundary condition per direction."""

    def __init__(self, handle, dom_lo, dom_hi, bc):
        self._h = C.c_void_p(handle)
        self.domain = Box(dom_lo, dom_hi)
        self.bc = tuple(int(b) for b in bc)

    @classmethod
    def chop(cls, dom_lo, dom_hi, max_box_size, bc=(L.DIRICHLET0,) * 3):
        h = C.c_void_p()
        L.check(L.lib().bxmg_define_boxarray(L.i32(dom_lo), L.i32(dom_hi), L.i32(bc), int(max_box_size), C.byref(h)))
        return cls(h.value, dom_lo, dom_hi, bc)

    @classmethod
    def from_boxes(cls, dom_lo, dom_hi, boxes, bc=(L.DIRICHLET0,) * 3):
        flat = []
        for b in boxes:
            b = b if isinstance(b, Box) else Box(*b)
            flat += list(b.small) + list(b.big)
        h = C.c_void_p()
        L.check(L.lib().bxmg_define_boxarray_list(L.i32(dom_lo), L.i32(dom_hi), L.i32(bc), len(boxes), L.i32(flat),
                                                  C.byref(h)))
        return cls(h.value, dom_lo, dom_hi, bc)

    @property
    def periodic(self):
        return tuple(int(b == L.PERIODIC) for b in self.bc)

    def __len__(self):
        n = C.c_int32()
        L.check(L.lib().bxmg_boxarray_get(self._h, C.byref(n), None))
        return n.value

    @property
    def boxes(self):
        n = len(self)
        arr = (C.c_int32 * (6 * n))()
        cnt = C.c_int32()
        L.check(L.lib().bxmg_boxarray_get(self._h, C.byref(cnt), arr))
        return [Box(arr[6 * b:6 * b + 3], arr[6 * b + 3:6 * b + 6]) for b in range(n)]

    def hierarchy(self):
        """[(domain Box, [boxes])] of the multigrid levels the solver builds."""
        capl, capb = 64, 40 * len(self) + 64
        nl = C.c_int32()
        nb = (C.c_int32 * capl)()
        dom = (C.c_int32 * (6 * capl))()
        lh = (C.c_int32 * (6 * capb))()
        L.check(L.lib().bxmg_boxarray_hierarchy(self._h, capl, C.byref(nl), nb, dom, capb, lh))
        out, o = [], 0
        for l in range(nl.value):
            bl = []
            for _ in range(nb[l]):
                bl.append(Box(lh[6 * o:6 * o + 3], lh[6 * o + 3:6 * o + 6]))
                o += 1
            out.append((Box(dom[6 * l:6 * l + 3], dom[6 * l + 3:6 * l + 6]), bl))
        return out

    def __del__(self):
        try:
            if self._h:
                L.lib().bxmg_boxarray_release(self._h)
                self._h = None
        except Exception:
            pass


# ------------------------------------------------------------------- Context
class Context:
    """A HIP device plus the stream the library enqueues on (torch's current
    stream by default)."""

    def __init__(self, device=0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        h = C.c_void_p()
        L.check(L.lib().bxmg_ctx_create(int(device), C.c_void_p(stream.cuda_stream), C.byref(h)))
        self._h = h

    def tune(self, param, value):
        """One launch-shape knob (bxmg_ctx_tune); applies to hierarchies and
        batch plans built afterwards."""
        L.check(L.lib().bxmg_ctx_tune(self._h, int(param), int(value)))

    def set_launch_shape(self, planes_per_thread, buffer_addressing, tile_rows_log2_cap):
        """Knobs 0 and 1 (planes per thread), 2 (32-bit buffer offsets) and 3
        (log2 of the tile-row cap) together."""
        for param, value in ((0, planes_per_thread), (1, planes_per_thread), (2, buffer_addressing),
                             (3, tile_rows_log2_cap)):
            self.tune(param, value)

    def close(self):
        if self._h:
            L.lib().bxmg_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx = None


def default_context():
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context(0)
    return _default_ctx


# ------------------------------------------------------------------ MultiFab
class MultiFab:
    """Data on every box of a BoxArray grown by nghost, one device slab in a
    torch buffer; box b is F-order (x, y, z, component)."""

    def __init__(self, ba: BoxArray, ncomp=1, nghost=1, dtype="f64", ctx: Context | None = None):
        import torch
        self.ctx = ctx or default_context()
        self.ba = ba
        self.ncomp, self.nghost = int(ncomp), int(nghost)
        self.dtype = dtype
        code = L.F64 if dtype == "f64" else L.F32
        self.torch_dtype = torch.float64 if dtype == "f64" else torch.float32
        nbytes = L.lib().bxmg_multifab_bytes(ba._h, self.ncomp, self.nghost, code)
        if nbytes == 0:
            raise L.BxmgError(-1, "bad MultiFab parameters")
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda:%d" % self.ctx.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.bytes = nbytes
        self.slab = raw[off:off + nbytes].view(self.torch_dtype)  # flat typed view of the whole slab
        h = C.c_void_p()
        L.check(L.lib().bxmg_alloc_multifab(self.ctx._h, ba._h, self.ncomp, self.nghost, code,
                                            C.c_void_p(self.slab.data_ptr()), C.byref(h)))
        self._h = h
        self._views = None

    @property
    def n_grow_vect(self):
        return (self.nghost,) * 3

    def __len__(self):
        return len(self.ba)

    def _box_views(self):
        if self._views is None:
            es = self.slab.element_size()
            base = self.slab.data_ptr()
            out = []
            for b in range(len(self.ba)):
                p = C.c_void_p()
                lo = (C.c_int32 * 3)()
                hi = (C.c_int32 * 3)()
                st = (C.c_int64 * 4)()
                L.check(L.lib().bxmg_multifab_box_view(self._h, b, C.byref(p), lo, hi, st))
                out.append(((p.value - base) // es, tuple(lo), tuple(hi), tuple(st)))
            self._views = out
        return self._views

    def array(self, b, order="F"):
        """Zero-copy torch view of box b (grown).  order "F": indices
        (x, y, z[, comp]) with x unit stride; order "C": (comp, z, y, x)."""
        import torch
        off, lo, hi, st = self._box_views()[b]
        shape = tuple(hi[d] - lo[d] + 1 for d in range(3))
        v = torch.as_strided(self.slab, shape + (self.ncomp,), st[:3] + (st[3],), off)
        if order == "C":
            return v.permute(3, 2, 1, 0)
        return v if self.ncomp > 1 else v[..., 0]

    def grown_box(self, b):
        off, lo, hi, st = self._box_views()[b]
        return Box(lo, hi)

    def set_val(self, v):
        self.slab.fill_(v)
        return self

    # -- host copies (tests, examples) -------------------------------------
    def from_global(self, glob, ghost=None, comp=0):
        """Set valid cells of component comp from a domain-sized F-order array;
        ghost cells become `ghost` (if not None)."""
        import torch
        host = self.slab.cpu().numpy().copy()
        dlo = self.ba.domain.small
        for b, (off, lo, hi, st) in enumerate(self._box_views()):
            shape = tuple(hi[d] - lo[d] + 1 for d in range(3))
            n = shape[0] * shape[1] * shape[2]
            v = host[off + comp * st[3]: off + comp * st[3] + n].reshape(shape, order="F")
            if ghost is not None:
                v[...] = ghost
            ng = self.nghost
            s = tuple(slice(lo[d] + ng - dlo[d], hi[d] - ng - dlo[d] + 1) for d in range(3))
            v[ng:shape[0] - ng, ng:shape[1] - ng, ng:shape[2] - ng] = glob[s]
        self.slab.copy_(torch.from_numpy(host))
        return self

    def from_tensor(self, t, comp=0):
        """Set valid cells of component comp from a domain-sized device tensor
        indexed [i, j, k] (box by box, on the device)."""
        D = self.ba.domain
        ng = self.nghost
        for b in range(len(self.ba)):
            g = self.grown_box(b)
            v = self.array(b)
            if self.ncomp > 1:
                v = v[..., comp]
            src = t[tuple(slice(g.small[d] + ng - D.small[d], g.big[d] - ng - D.small[d] + 1) for d in range(3))]
            v[ng:v.shape[0] - ng, ng:v.shape[1] - ng, ng:v.shape[2] - ng].copy_(src)
        return self

    def copy_host(self, glob, to_device, comp=0):
        """bxmg_multifab_copy_host: valid cells of component comp <-> a
        domain-sized F-order numpy array of the MultiFab's dtype."""
        dt = np.float64 if self.dtype == "f64" else np.float32
        assert glob.dtype == dt and glob.flags.f_contiguous and glob.shape == self.ba.domain.size
        L.check(L.lib().bxmg_multifab_copy_host(self._h, 1 if to_device else 0, glob.ctypes.data_as(C.c_void_p),
                                                int(comp), C.c_void_p(self.ctx.stream.cuda_stream)))
        return glob

    def from_packed(self, packed):
        """Set all cells (valid + ghost) from the oracle's packed layout."""
        import torch
        host = self.slab.cpu().numpy().copy()
        o = 0
        for off, lo, hi, st in self._box_views():
            n = int(np.prod([hi[d] - lo[d] + 1 for d in range(3)])) * self.ncomp
            host[off:off + n] = packed[o:o + n]
            o += n
        self.slab.copy_(torch.from_numpy(host))
        return self

    def to_packed(self):
        host = self.slab.cpu().numpy()
        parts = []
        for off, lo, hi, st in self._box_views():
            n = int(np.prod([hi[d] - lo[d] + 1 for d in range(3)])) * self.ncomp
            parts.append(host[off:off + n])
        return np.ascontiguousarray(np.concatenate(parts))

    def to_global(self, comp=0):
        host = self.slab.cpu().numpy()
        D = self.ba.domain
        out = np.full(D.size, np.nan, dtype=host.dtype, order="F")
        ng = self.nghost
        for off, lo, hi, st in self._box_views():
            shape = tuple(hi[d] - lo[d] + 1 for d in range(3))
            n = shape[0] * shape[1] * shape[2]
            v = host[off + comp * st[3]: off + comp * st[3] + n].reshape(shape, order="F")
            s = tuple(slice(lo[d] + ng - D.small[d], hi[d] - ng - D.small[d] + 1) for d in range(3))
            out[s] = v[ng:shape[0] - ng, ng:shape[1] - ng, ng:shape[2] - ng]
        return out

    # -- communication -----------------------------------------------------
    def fill_boundary(self, scomp=0, ncomp=None, cross=False, stream=None):
        ncomp = self.ncomp - scomp if ncomp is None else ncomp
        s = (stream or self.ctx.stream).cuda_stream
        L.check(L.lib().bxmg_fill_boundary(self._h, scomp, ncomp, int(bool(cross)), C.c_void_p(s)))
        return self

    def parallel_copy(self, src, scomp=0, dcomp=0, ncomp=None, nghost=0, stream=None):
        """ParallelCopy from src (another decomposition of the same domain)
        into this MultiFab's cells grown by nghost."""
        ncomp = min(self.ncomp - dcomp, src.ncomp - scomp) if ncomp is None else ncomp
        s = (stream or self.ctx.stream).cuda_stream
        L.check(L.lib().bxmg_parallel_copy(self._h, int(dcomp), src._h, int(scomp), int(ncomp), int(nghost),
                                           C.c_void_p(s)))
        return self

    def apply_domain_bc(self, scomp=0, ncomp=None, odd=True, stream=None):
        ncomp = self.ncomp - scomp if ncomp is None else ncomp
        s = (stream or self.ctx.stream).cuda_stream
        L.check(L.lib().bxmg_apply_domain_bc(self._h, scomp, ncomp, int(bool(odd)), C.c_void_p(s)))
        return self

    def close(self):
        if getattr(self, "_h", None):
            L.lib().bxmg_multifab_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
