"""GPU tests of the batch engine (many problems in one set of launches).

The bar: each problem's batched result is bitwise the result of solving it
alone (the same kernels in the same order per problem, stop tests on exact
max-norms), and every batched solution meets its tolerance as recomputed by
the oracle's FP64 operator.  The hipGraph-captured cycle is checked against
stage-by-stage launches over several steps (every replay's residual norm is
in the history, and the solutions must agree bitwise).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

MB = 1 << 20


@pytest.fixture(scope="module")
def bx():
    import paper_2403_12179_amd as bx
    return bx


def problem(bx, n, per, seed, var=False, mb=32):
    bc = (bx.PERIODIC if per else bx.DIRICHLET0,) * 3
    ba = bx.BoxArray.chop((0, 0, 0), (n - 1,) * 3, mb, bc=bc)
    f = W.uniform_rhs((n, n, n), seed, mean_zero=per)
    beta = W.smooth_gaussian_beta((n, n, n), seed + 1) if var else None
    phi = bx.MultiFab(ba).set_val(0.0)
    rhs = bx.MultiFab(ba).set_val(0.0).from_global(f)
    bmf = bx.MultiFab(ba).set_val(1.0).from_global(beta) if var else None
    return dict(n=n, per=per, ba=ba, f=f, beta=beta, phi=phi, rhs=rhs, bmf=bmf)


def run_batch(bx, probs, budget=512 * MB, graph=True, chunk=2, var=False, **params):
    b = bx.Batch(probs[0]["phi"].ctx, budget, 64, var=var, graph=graph, **params)
    ids = {}
    for q, p in enumerate(probs):
        pid = b.add(p["phi"], p["rhs"], p["bmf"])
        assert pid is not None
        ids[pid] = q
    out = {ids[i]: r for i, r in b.run(chunk)}
    b.close()
    return out


def solve_alone(bx, p, **params):
    p["phi"].set_val(0.0)
    res = bx.mlmg_solve(p["phi"], p["rhs"], p["bmf"], **params)
    return p["phi"].to_global(), res


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_alone_periodic(bx, precision):
    """Batched periodic problems of uneven size (boxes of 32 and 16, bottoms
    2^3 and 3^3) are bitwise their lone solves, cycles and history included."""
    probs = [problem(bx, n, True, 4000 + q) for q, n in enumerate([32, 48, 64, 32, 96])]
    alone = [solve_alone(bx, p, precision=precision) for p in probs]
    for p in probs:
        p["phi"].set_val(0.0)
    res = run_batch(bx, probs, precision=precision)
    assert sorted(res) == list(range(len(probs)))
    for q, p in enumerate(probs):
        u_alone, r_alone = alone[q]
        r = res[q]
        assert r.ok and r_alone.ok
        assert r.cycles == r_alone.cycles
        assert r.hist == r_alone.hist
        assert np.array_equal(p["phi"].to_global(), u_alone), q


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_var_dirichlet_equals_alone(bx, orc, precision):
    probs = [problem(bx, n, False, 6000 + q, var=True) for q, n in enumerate([32, 64, 48])]
    alone = [solve_alone(bx, p, precision=precision) for p in probs]
    for p in probs:
        p["phi"].set_val(0.0)
    res = run_batch(bx, probs, var=True, precision=precision)
    for q, p in enumerate(probs):
        u = p["phi"].to_global()
        assert res[q].ok and res[q].cycles == alone[q][1].cycles
        assert np.array_equal(u, alone[q][0]), q
        if precision == 0:  # max norms are exact, whichever kernel took them
            assert res[q].hist == alone[q][1].hist, q
        n = p["n"]
        r = p["f"] - orc.apply_op((0, 0, 0), (n - 1,) * 3, (0, 0, 0), 1.0 / n, u, p["beta"])
        assert np.max(np.abs(r)) <= 1e-10 * np.max(np.abs(p["f"]))


def test_batch_matches_oracle(bx, orc):
    """FP64 batch of Dirichlet and periodic problems against oracle solves."""
    probs = [problem(bx, 32, False, 11), problem(bx, 48, True, 12), problem(bx, 64, False, 13, mb=16)]
    res = run_batch(bx, probs)
    for q, p in enumerate(probs):
        n, per = p["n"], (1, 1, 1) if p["per"] else (0, 0, 0)
        u = p["phi"].to_global()
        r = p["f"] - orc.apply_op((0, 0, 0), (n - 1,) * 3, per, 1.0 / n, u)
        assert np.max(np.abs(r)) <= 1e-10 * np.max(np.abs(p["f"]))
        uo, io = orc.solve((0, 0, 0), (n - 1,) * 3, per, [(b.small, b.big) for b in p["ba"].boxes], p["f"])
        assert abs(res[q].cycles - io["cycles"]) <= 1
        assert np.max(np.abs(u - uo)) <= 0.405 * n * n * 2e-10 * np.max(np.abs(uo))


def test_graph_replays_equal_stage_launches(bx):
    """One step per replay with the host's finish work in between: histories
    (one entry per replay) and solutions are bitwise those of the eager run."""
    out = []
    for graph in (True, False):
        probs = [problem(bx, n, True, 7000 + q) for q, n in enumerate([32, 64, 48])]
        res = run_batch(bx, probs, graph=graph, chunk=1, precision=1)
        out.append(([p["phi"].to_global() for p in probs], res))
    for q in range(3):
        assert np.array_equal(out[0][0][q], out[1][0][q])
        assert out[0][1][q].hist == out[1][1][q].hist
        assert len(out[0][1][q].hist) >= 4


def test_admission_by_footprint_and_continuous_add(bx):
    p1, p2 = problem(bx, 64, True, 31), problem(bx, 64, True, 32)
    b = bx.Batch(p1["phi"].ctx, 64 * MB, 8)
    need = b.footprint(p1["ba"])
    assert need > 0
    b.close()
    # room for one problem only: the second waits until the first finishes
    b = bx.Batch(p1["phi"].ctx, int(need * 1.5), 8)
    id1 = b.add(p1["phi"], p1["rhs"])
    assert id1 is not None
    assert b.add(p2["phi"], p2["rhs"]) is None
    st = b.stats()
    assert st["running"] == 1 and st["bytes_used"] <= st["bytes_budget"]
    done = b.run(2)
    assert [i for i, _ in done] == [id1]
    id2 = b.add(p2["phi"], p2["rhs"])
    assert id2 is not None
    done = b.run(2)
    assert [i for i, _ in done] == [id2] and done[0][1].ok
    b.close()
    u1, _ = solve_alone(bx, p1)
    p1["phi"].set_val(0.0)
    b = bx.Batch(p1["phi"].ctx, 256 * MB, 8)
    b.add(p1["phi"], p1["rhs"])
    # a problem admitted while another is mid-solve (from a zero guess, as
    # the lone solve below)
    b.step(2)
    p2["phi"].set_val(0.0)
    b.add(p2["phi"], p2["rhs"])
    b.run(1)
    assert np.array_equal(p1["phi"].to_global(), u1)
    u2 = p2["phi"].to_global()
    assert np.array_equal(u2, solve_alone(bx, p2)[0])
    b.close()


def test_status_codes_and_remove(bx):
    b = bx.Batch(bx.default_context(), 128 * MB, 8, max_cycles=2, rel_tol=1e-14)
    p = problem(bx, 32, False, 41)
    pid = b.add(p["phi"], p["rhs"])
    done = b.run(4)
    assert done[0][0] == pid and done[0][1].status == -4 and done[0][1].cycles == 2
    b.close()
    b = bx.Batch(bx.default_context(), 128 * MB, 8)
    bad = p["f"].copy()
    bad[3, 4, 5] = np.inf
    p["rhs"].from_global(bad)
    b.add(p["phi"], p["rhs"])
    assert b.step(1) == 0  # the admission check on the device retires it at once
    done = b.poll()
    assert done[0][1].status == -5 and done[0][1].cycles == 0
    p["rhs"].set_val(0.0)
    p["phi"].set_val(0.0)
    b.add(p["phi"], p["rhs"])
    assert b.step(1) == 0
    done = b.poll()
    assert done[0][1].ok and done[0][1].cycles == 0 and not np.any(p["phi"].to_global())
    q = problem(bx, 32, True, 42)
    qid = b.add(q["phi"], q["rhs"])
    b.remove(qid)
    assert b.step(1) == 0 and b.poll() == []
    with pytest.raises(bx.BxmgError):
        b.remove(12345)
    with pytest.raises(bx.BxmgError):
        b.add(q["phi"], q["rhs"], q["phi"])  # beta in a constant-coefficient batch
    b.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_grouped_admission_and_retirement(bx, precision):
    """Problems added together are admitted by one group of launches and the
    ones that stop together are converted back by one: periodic and Dirichlet
    problems of several shapes in one group (the periodic means taken for a
    subset of the group), a zero right-hand side, a problem removed before
    the step that would admit it, and more problems joining a running batch.
    Every result is bitwise its lone solve, history included."""
    shapes = [(32, True, 32), (48, False, 32), (64, True, 16), (32, False, 32), (96, True, 32), (64, False, 32)]
    probs = [problem(bx, n, per, 8100 + q, mb=mb) for q, (n, per, mb) in enumerate(shapes)]
    zero = problem(bx, 32, True, 8199)
    zero["rhs"].set_val(0.0)
    gone = problem(bx, 48, True, 8198)
    alone = [solve_alone(bx, p, precision=precision) for p in probs]
    for p in probs + [zero, gone]:
        p["phi"].set_val(0.0)
    b = bx.Batch(probs[0]["phi"].ctx, 512 * MB, 64, precision=precision)
    ids = {}
    for q, p in enumerate(probs[:4]):
        ids[b.add(p["phi"], p["rhs"])] = q
    idz = b.add(zero["phi"], zero["rhs"])
    idg = b.add(gone["phi"], gone["rhs"])
    b.remove(idg)  # before any launch: never admitted
    b.step(1)
    for q, p in enumerate(probs[4:], start=4):  # join the running batch
        ids[b.add(p["phi"], p["rhs"])] = q
    done = dict(b.run(2))
    b.close()
    assert idg not in done and sorted(done) == sorted(list(ids) + [idz])
    assert done[idz].ok and done[idz].cycles == 0
    assert np.all(zero["phi"].to_global() == 0.0)
    for i, q in ids.items():
        u_alone, r_alone = alone[q]
        assert done[i].ok and done[i].cycles == r_alone.cycles, q
        assert done[i].hist == r_alone.hist, q
        assert np.array_equal(probs[q]["phi"].to_global(), u_alone), q


@pytest.mark.parametrize("precision", [0, 1])
def test_zero_guess_flag_per_problem(bx, orc, precision):
    """A problem's first residual skips the reads of its guess only when that
    guess is +0.0 in every cell (one flag per slot, cleared at admission).
    In one batch: a +0.0 guess and a -0.0 guess of the same problem (the
    second takes the full path) end with the same history and solution, and
    a guess that is zero but for one cell has the oracle operator's residual
    of it as hist[0].  A second pass in the reverse order puts each guess in
    another problem's former slot."""
    n = 32
    probs = [problem(bx, n, False, 4100) for _ in range(3)]
    g = np.zeros((n, n, n), order="F")
    g[3, n // 2, 7] = 0.25
    f = probs[0]["f"]
    r = f - orc.apply_op((0, 0, 0), (n - 1,) * 3, (0, 0, 0), 1.0 / n, g, None)
    want0 = np.abs(r).max() / np.abs(f).max()
    b = bx.Batch(probs[0]["phi"].ctx, 512 * MB, 64, precision=precision)
    try:
        for order in ([0, 1, 2], [2, 1, 0]):
            probs[0]["phi"].set_val(0.0)
            probs[1]["phi"].set_val(-0.0)
            probs[2]["phi"].set_val(0.0).from_global(g)
            ids = {}
            for q in order:
                pid = b.add(probs[q]["phi"], probs[q]["rhs"], None)
                assert pid is not None
                ids[pid] = q
            out = {ids[i]: res for i, res in b.run(2)}
            assert sorted(out) == [0, 1, 2] and all(out[q].ok for q in out)
            assert out[0].hist == out[1].hist
            assert np.array_equal(probs[0]["phi"].to_global(), probs[1]["phi"].to_global())
            assert out[2].hist[0] == pytest.approx(want0, rel=1e-14)
    finally:
        b.close()
