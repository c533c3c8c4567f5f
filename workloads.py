"""Seeded synthetic inputs shaped like the multigrid workloads.

This module holds input generation only (random fields, manufactured
right-hand sides, size draws): none of the solver's arithmetic.  Both the HIP
path's tests/benchmark and the oracle consume it.  All draws use numpy's
PCG64 ``default_rng(seed)``; fields are generated over the global domain in
F-order (x fastest) so they do not depend on the box decomposition.
"""
from __future__ import annotations

import numpy as np


def cell_centres(n, lo=0, h=None):
    h = 1.0 / n if h is None else h
    return (np.arange(lo, lo + n) + 0.5) * h


def sine_rhs(n, periodic=True):
    """Manufactured RHS on the unit cube with cubic cells h = 1/n.

    periodic : f = -3 (2 pi)^2 sin(2 pi x) sin(2 pi y) sin(2 pi z)
    Dirichlet: f = -3 pi^2     sin(pi x)   sin(pi y)   sin(pi z)
    Returns (f, s) with s the sine product at the cell centres.
    """
    x = cell_centres(n)
    k = 2.0 * np.pi if periodic else np.pi
    sx = np.sin(k * x)
    s = sx[:, None, None] * sx[None, :, None] * sx[None, None, :]
    return np.asfortranarray(-3.0 * k * k * s), np.asfortranarray(s)


def uniform_rhs(shape, seed, mean_zero=False):
    """i.i.d. uniform[-1, 1] over the global domain (F-order draw order)."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    f = rng.uniform(-1.0, 1.0, size=n).reshape(shape, order="F")
    if mean_zero:
        f = f - f.mean()
    return np.asfortranarray(f)


def smooth_gaussian_beta(shape, seed, passes=3):
    """beta = exp(g): g0 ~ N(0,1) i.i.d., `passes` periodic 3x3x3 box-filter
    passes, then standardised to mean 0 and (population) std 1."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    g = rng.standard_normal(n).reshape(shape, order="F")
    for _ in range(passes):
        acc = np.zeros_like(g)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    acc += np.roll(g, (dx, dy, dz), axis=(0, 1, 2))
        g = acc / 27.0
    g = (g - g.mean()) / g.std()
    return np.asfortranarray(np.exp(g))


# ------------------------------------------------------------------------
# Device-side draws of the same distributions (torch's Philox generator on
# the GPU, seeded per field), for workloads too large to draw and copy from
# the host in a benchmark: the recipes are those of uniform_rhs and
# smooth_gaussian_beta, the random streams are not.  Tensors are indexed
# [i, j, k] like the numpy fields.


def uniform_rhs_device(shape, seed, mean_zero=False, device="cuda"):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f = torch.rand(tuple(shape), generator=g, device=device, dtype=torch.float64) * 2.0 - 1.0
    if mean_zero:
        f = f - f.mean()
    return f


def smooth_gaussian_beta_device(shape, seed, passes=3, device="cuda"):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    x = torch.randn(tuple(shape), generator=g, device=device, dtype=torch.float64)
    for _ in range(passes):
        acc = torch.zeros_like(x)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    acc += torch.roll(x, (dx, dy, dz), dims=(0, 1, 2))
        x = acc / 27.0
    x = (x - x.mean()) / x.std(unbiased=False)
    return torch.exp(x)


def dyadic_codes(shape, seed=0, scale=1.0 / 64):
    """Exactly representable small codes: integers in [-64, 64] times `scale`
    (a power of two), so sums of up to 64 of them with weights k/64 are exact
    in FP64 and FP32."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.integers(-64, 65, size=shape).astype(np.float64) * scale)


def batch_edges(nprob, seed, choices=(32, 48, 64, 96, 128)):
    """Cube edges of a batch of independent problems, uniform over choices."""
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.choice(np.asarray(choices), size=nprob)]


def serving_trace(nreq, seed, rate=200.0, lo=32, hi=256, step=16):
    """Open-loop request trace: exponential inter-arrivals (mean 1/rate s),
    edge = clamp(step*round(exp(U(ln lo, ln hi))/step), lo, hi), tolerance
    10^U(-10, -8), coefficient kind Bernoulli(1/2) (0 constant, 1 lognormal)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=nreq))
    e = np.exp(rng.uniform(np.log(lo), np.log(hi), size=nreq))
    edges = np.clip(step * np.round(e / step), lo, hi).astype(int)
    tols = 10.0 ** rng.uniform(-10.0, -8.0, size=nreq)
    kinds = rng.integers(0, 2, size=nreq)
    return [dict(t=float(t[q]), edge=int(edges[q]), tol=float(tols[q]), kind=int(kinds[q]), seed=5000 + q)
            for q in range(nreq)]


def composite_layout(n, kind="centre", max_box=32):
    """Two-level layout on a coarse n^3 domain: (coarse boxes, fine boxes),
    fine boxes in fine indices (refinement ratio 2).
      centre : the central half of the domain refined ([n/4, 3n/4) coarse
               cells), chopped into fine boxes of edge max_box
      holed  : the same boxes less the last one (their union is no rectangle)
      lshape : an L of two abutting fine boxes plus a detached one
    Coarse boxes: the domain chopped into boxes of edge min(n, 32)."""
    cb = chop_boxes(n, min(n, 32))
    if kind == "centre":
        q = n // 4
        lo, hi = 2 * q, 2 * (n - q)
        fb = []
        for k in range(lo, hi, max_box):
            for j in range(lo, hi, max_box):
                for i in range(lo, hi, max_box):
                    fb.append(((i, j, k), (min(i + max_box, hi) - 1, min(j + max_box, hi) - 1,
                                           min(k + max_box, hi) - 1)))
        return cb, fb
    if kind == "holed":  # the central half in boxes of max_box, less its last box: not one rectangle
        q = n // 4
        lo, hi = 2 * q, 2 * (n - q)
        fb = []
        for k in range(lo, hi, max_box):
            for j in range(lo, hi, max_box):
                for i in range(lo, hi, max_box):
                    fb.append(((i, j, k), (min(i + max_box, hi) - 1, min(j + max_box, hi) - 1,
                                           min(k + max_box, hi) - 1)))
        return cb, fb[:-1]
    if kind == "lshape":
        a = n // 4
        return cb, [((2 * a, 2 * a, 2 * a), (4 * a - 1, 4 * a - 1, 4 * a - 1)),
                    ((4 * a, 2 * a, 2 * a), (5 * a - 1, 3 * a - 1, 4 * a - 1)),
                    ((5 * a, 5 * a, 5 * a), (6 * a - 1, 6 * a - 1, 6 * a - 3))]
    raise ValueError(kind)


def chop_boxes(n, edge):
    """The cube [0, n)^3 cut into boxes of the given edge (last one ragged)."""
    out = []
    for k in range(0, n, edge):
        for j in range(0, n, edge):
            for i in range(0, n, edge):
                out.append(((i, j, k), (min(i + edge, n) - 1, min(j + edge, n) - 1, min(k + edge, n) - 1)))
    return out


def fine_mask(n, fine_boxes):
    """Boolean (2n)^3 mask of the fine cells inside the fine boxes."""
    m = np.zeros((2 * n,) * 3, bool)
    for lo, hi in fine_boxes:
        m[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1] = True
    return m
