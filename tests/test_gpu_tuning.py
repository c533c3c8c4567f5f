"""GPU tests of the launch-shape tuner with its JSON cache: a batch tuned on
its own context times every candidate once and then comes from the cache;
lone solves likewise; the tuned shape changes no result (the batch's
solutions under the tuned and the default shape are bitwise equal, and equal
to the lone FP64/mixed solves, which the batch tests tie to the oracle)."""
import json

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bx():
    import paper_2403_12179_amd as bx
    return bx


def problems(bx, ctx, edges):
    out = []
    for q, n in enumerate(edges):
        ba = bx.BoxArray.chop((0, 0, 0), (n - 1,) * 3, 16, bc=(bx.PERIODIC,) * 3)
        f = W.uniform_rhs((n, n, n), 7100 + q, mean_zero=True)
        phi = bx.MultiFab(ba, ctx=ctx).set_val(0.0)
        rhs = bx.MultiFab(ba, ctx=ctx).set_val(0.0).from_global(f)
        out.append((phi, rhs, None, 1e-10))
    return out


def batch_solutions(bx, ctx, probs):
    b = bx.Batch(ctx, 256 << 20, 64, precision=1)
    ids = {}
    for q, (phi, rhs, beta, tol) in enumerate(probs):
        phi.set_val(0.0)
        ids[b.add(phi, rhs, beta, rel_tol=tol)] = q
    res = {ids[i]: r for i, r in b.run(2)}
    b.close()
    return [probs[q][0].to_global() for q in range(len(probs))], [res[q] for q in range(len(probs))]


def test_tune_batch_then_cache(bx, tmp_path):
    from paper_2403_12179_amd import tuning
    ctx = bx.Context(0)
    probs = problems(bx, ctx, [16, 24, 32, 16, 48])
    path = str(tmp_path / "tune.json")
    print("tune_batch: timing every candidate", flush=True)
    first = tuning.tune_batch(ctx, probs, 256 << 20, 64, cache=path, reps=1, precision=1)
    assert first["source"] == "timed" and first["candidates"] == 24
    assert first["seconds_per_batch"] <= first["default_shape_seconds"]
    shape = {k: first[k] for k in tuning.DEFAULT_SHAPE}
    assert shape in tuning.candidates()
    stored = json.load(open(path))
    assert list(stored) == [first["key"]]
    assert first["key"].split("|")[1:4] == ["batch", "f32-in-f64", "const"]
    second = tuning.tune_batch(ctx, probs, 256 << 20, 64, cache=path, precision=1)
    assert second["source"] == "cache" and {k: second[k] for k in tuning.DEFAULT_SHAPE} == shape
    # another arithmetic is another entry
    third = tuning.tune_batch(ctx, probs[:2], 256 << 20, 64, cache=False, reps=1, precision=0)
    assert third["source"] == "timed" and len(json.load(open(path))) == 1
    # results do not depend on the shape
    tuning.apply(ctx, shape)
    u_t, r_t = batch_solutions(bx, ctx, probs)
    tuning.apply(ctx, tuning.DEFAULT_SHAPE)
    u_d, r_d = batch_solutions(bx, ctx, probs)
    for a, b, ra, rb in zip(u_t, u_d, r_t, r_d):
        assert ra.ok and rb.ok and ra.cycles == rb.cycles and ra.hist == rb.hist
        assert np.array_equal(a, b)


def test_tune_solve_then_cache(bx, tmp_path):
    from paper_2403_12179_amd import tuning
    ctx = bx.Context(0)
    phi, rhs, _, _ = problems(bx, ctx, [32])[0]
    path = str(tmp_path / "tune.json")
    first = tuning.tune_solve(bx.MultiFab(phi.ba, ctx=ctx), rhs, cache=path, cycles=1)
    assert first["source"] == "timed" and first["candidates"] == 24
    second = tuning.tune_solve(bx.MultiFab(phi.ba, ctx=ctx), rhs, cache=path)
    assert second["source"] == "cache" and second["key"] == first["key"]
    assert all(second[k] == first[k] for k in tuning.DEFAULT_SHAPE)
    assert first["key"].split("|")[1:6] == ["solve", "f64", "const", "dom32x32x32/b8/e16", "PPP"]
    res = bx.mlmg_solve(phi, rhs, rel_tol=1e-10)
    assert res.ok
