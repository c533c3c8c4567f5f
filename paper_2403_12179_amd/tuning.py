"""Launch-shape tuning with a persistent cache.

The library's kernels take their work decomposition from four context knobs
(planes per thread, 32-bit buffer addressing, the tile-row cap; see
bxmg_ctx_tune).  The best setting depends on the workload: a lone solve on
one large merged box wants different tiles from a batch of many small
problems.  This module times the candidates on the caller's own workload,
keeps the winner in a JSON file keyed by what decides it (GPU architecture,
solve form, arithmetic, coefficient kind, domain, box edge, boundaries), and
applies a cached entry without timing on later runs.

Results never depend on the knobs (the solver's iterates are bitwise the same
under every setting), so a stale or foreign cache entry costs only speed.

The cache file is BXMG_TUNE_CACHE if set, else ~/.cache/bxmg/tune.json; pass
cache=False to time without reading or writing it."""
from __future__ import annotations

import functools
import hashlib
import json
import os
import tempfile
import time

from . import _lib as L
from . import solver as S

# the candidate grid the native autotuner also walks: planes per thread,
# log2 tile-row cap, 32-bit buffer addressing
PLANES = (1, 2, 4, 8)
ROWS_LOG2 = (2, 3, 8)
ADDRESSING = (1, 0)
DEFAULT_SHAPE = {"planes_per_thread": 4, "buffer_addressing": 1, "tile_rows_log2_cap": 8}
FORMAT = 1


def candidates():
    return [{"planes_per_thread": z, "buffer_addressing": r, "tile_rows_log2_cap": ly}
            for z in PLANES for ly in ROWS_LOG2 for r in ADDRESSING]


def default_cache_path():
    p = os.environ.get("BXMG_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "bxmg", "tune.json")


class TuneCache:
    """A JSON file {key: entry}; every put() rewrites it atomically (a
    temporary file in the same folder, then a rename), so readers never see
    a torn file.  Entries with another format number are ignored."""

    def __init__(self, path=None):
        self.path = path or default_cache_path()
        self._d = self._load()

    def _load(self):
        try:
            with open(self.path) as fh:
                d = json.load(fh)
        except (OSError, ValueError):
            return {}
        if not isinstance(d, dict):
            return {}
        return {k: v for k, v in d.items() if isinstance(v, dict) and v.get("format") == FORMAT}

    def get(self, key):
        return self._d.get(key)

    def put(self, key, entry):
        """Stores the entry; returns False (the entry kept in memory only)
        when the file cannot be written, e.g. a read-only home."""
        self._d = self._load()  # keep what other processes wrote meanwhile
        self._d[key] = dict(entry, format=FORMAT)
        folder = os.path.dirname(os.path.abspath(self.path))
        try:
            os.makedirs(folder, exist_ok=True)
            fd, tmp = tempfile.mkstemp(prefix=".tune.", dir=folder)
        except OSError:
            return False
        try:
            with os.fdopen(fd, "w") as fh:
                json.dump(self._d, fh, indent=1, sort_keys=True)
            os.replace(tmp, self.path)
        except BaseException:
            if os.path.exists(tmp):
                os.unlink(tmp)
            raise
        return True

    def __len__(self):
        return len(self._d)


def _arch(device):
    import torch
    name = getattr(torch.cuda.get_device_properties(device), "gcnArchName", "") or "unknown"
    return name.split(":")[0]


@functools.lru_cache(maxsize=None)
def lib_fingerprint():
    """First 12 hex digits of the built library's SHA-1: a rebuilt library
    (new kernels) gets fresh cache entries."""
    h = hashlib.sha1()
    with open(L.LIB_PATH, "rb") as fh:
        for chunk in iter(lambda: fh.read(1 << 20), b""):
            h.update(chunk)
    return h.hexdigest()[:12]


def _bc_code(bc):
    return "".join("P" if b == L.PERIODIC else "D" for b in bc)


def _arith(params):
    return "f32-in-f64" if int(params.get("precision", 0)) else "f64"


def _geometry(ba):
    """Domain extents, box count and the largest box edge of a BoxArray."""
    ext = tuple(ba.domain.size)
    edge = max(max(b.size) for b in ba.boxes)
    return ext, len(ba), edge


def make_key(arch, form, arith, coef, geometry, bc, extra=()):
    """Cache key: 'arch|form|arithmetic|coef|geometry|bc[|extra...]' with
    geometry written as 'dom<nx>x<ny>x<nz>/b<boxes>/e<largest box edge>' for
    one problem, or for a batch as the sorted multiset of its problems'
    '<nx>x<ny>x<nz>/b<boxes>/e<edge>:<count>' joined by commas; extra holds
    the library fingerprint."""
    parts = [arch, form, arith, coef, geometry, bc] + [str(x) for x in extra]
    return "|".join(parts)


def _geom_one(ba):
    ext, nb, edge = _geometry(ba)
    return "dom%dx%dx%d/b%d/e%d" % (ext + (nb, edge))


def _geom_many(bas):
    hist = {}
    for ba in bas:
        ext, nb, edge = _geometry(ba)
        k = "%dx%dx%d/b%d/e%d" % (ext + (nb, edge))
        hist[k] = hist.get(k, 0) + 1
    return ",".join("%s:%d" % (k, hist[k]) for k in sorted(hist))


def solve_key(phi, beta=None, **params):
    coef = "cell" if beta is not None else "const"
    if float(params.get("alpha", 0.0)) != 0.0:
        coef += "+alpha"
    form = "solve" + ("-pcg" if int(params.get("krylov", 0)) else "")
    return make_key(_arch(phi.ctx.device), form, _arith(params), coef, _geom_one(phi.ba), _bc_code(phi.ba.bc),
                    ("lib" + lib_fingerprint(),))


def batch_key(ctx, problems, **params):
    coefs = sorted({"cell" if p[2] is not None else "const" for p in problems})
    bcs = sorted({_bc_code(p[0].ba.bc) for p in problems})
    return make_key(_arch(ctx.device), "batch", _arith(params), "+".join(coefs), _geom_many(p[0].ba for p in problems),
                    "+".join(bcs), ("lib" + lib_fingerprint(),))


def _open(cache):
    if cache is False:
        return None
    if isinstance(cache, TuneCache):
        return cache
    return TuneCache(cache)


def apply(ctx, shape):
    ctx.set_launch_shape(shape["planes_per_thread"], shape["buffer_addressing"], shape["tile_rows_log2_cap"])


def tune_solve(phi, rhs, beta=None, cache=None, cycles=2, **params):
    """Launch shape for lone solves of this problem on phi's context: the
    cached entry if there is one, else the native autotuner's pick (which
    overwrites phi), stored.  The shape is left applied on the context.
    Returns the entry with 'source' = 'cache' or 'timed'."""
    tc = _open(cache)
    key = solve_key(phi, beta, **params)
    hit = tc.get(key) if tc is not None else None
    if hit is not None:
        apply(phi.ctx, hit)
        return dict(hit, source="cache", key=key)
    t0 = time.perf_counter()
    best = S.autotune(phi, rhs, beta, cycles=cycles, **params)
    entry = {k: best[k] for k in DEFAULT_SHAPE}
    entry.update(ms_per_cycle=best["ms_per_cycle"], candidates=best["candidates"],
                 tuning_seconds=time.perf_counter() - t0)
    if tc is not None:
        tc.put(key, entry)
    apply(phi.ctx, entry)
    return dict(entry, source="timed", key=key)


def time_batch(ctx, problems, shape, budget_bytes, max_problems, chunk=2, reps=2, **params):
    """Least seconds over `reps` timed passes of one batch of every problem
    under one launch shape, after an untimed pass on the same batch object
    (plans, graph capture).  problems: [(phi, rhs, beta, rel_tol)], every phi
    on ctx; each phi is zeroed before each pass."""
    import torch
    apply(ctx, shape)
    best = None
    b = S.Batch(ctx, budget_bytes, max_problems, var=any(p[2] is not None for p in problems), **params)
    try:
        for rep in range(reps + 1):
            for phi, rhs, beta, tol in problems:
                phi.set_val(0.0)
                if b.add(phi, rhs, beta, rel_tol=tol) is None:
                    raise L.BxmgError(-6, "tune_batch: the problems do not fit the batch budget")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            done = b.run(chunk)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            if len(done) != len(problems) or not all(r.ok for _, r in done):
                raise L.BxmgError(-4, "tune_batch: a problem did not converge")
            if rep > 0:
                best = t if best is None else min(best, t)
    finally:
        b.close()
    return best


def tune_batch(ctx, problems, budget_bytes, max_problems, cache=None, chunk=2, reps=2, **params):
    """Launch shape for batches of these problems on ctx: the cached entry if
    there is one, else every candidate timed on the whole batch (the fastest
    kept and stored).  problems: [(phi, rhs, beta, rel_tol)], all on ctx;
    their phi are overwritten.  Leaves the shape applied on ctx and returns
    the entry with 'source' = 'cache' or 'timed'."""
    tc = _open(cache)
    key = batch_key(ctx, problems, **params)
    hit = tc.get(key) if tc is not None else None
    if hit is not None:
        apply(ctx, hit)
        return dict(hit, source="cache", key=key)
    t0 = time.perf_counter()
    timed = []
    for shape in candidates():
        timed.append((time_batch(ctx, problems, shape, budget_bytes, max_problems, chunk, reps, **params), shape))
    t_best, shape = min(timed, key=lambda x: x[0])
    t_default = next(t for t, s in timed if s == DEFAULT_SHAPE)
    entry = dict(shape, seconds_per_batch=t_best, default_shape_seconds=t_default, candidates=len(timed),
                 problems=len(problems), tuning_seconds=time.perf_counter() - t0)
    if tc is not None:
        tc.put(key, entry)
    apply(ctx, entry)
    return dict(entry, source="timed", key=key)
