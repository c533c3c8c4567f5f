"""GPU test of the continuous-batching server: requests of uneven size, both
coefficient kinds and different tolerances arrive while others are being
solved; each served result must be bitwise the result of solving that
request alone with the same parameters, and meet its tolerance as
recomputed by the oracle's FP64 operator."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bx():
    import paper_2403_12179_amd as bx
    return bx


def test_served_equals_alone(bx, orc):
    trace = W.serving_trace(10, 55, lo=32, hi=64)
    reqs = []
    for q in trace:
        e = q["edge"]
        ba = bx.BoxArray.chop((0, 0, 0), (e - 1,) * 3, 32, bc=(bx.DIRICHLET0,) * 3)
        f = W.uniform_rhs((e, e, e), q["seed"])
        beta = W.smooth_gaussian_beta((e, e, e), q["seed"] + 1) if q["kind"] else None
        reqs.append(dict(q=q, f=f, beta=beta, phi=bx.MultiFab(ba).set_val(0.0),
                         rhs=bx.MultiFab(ba).set_val(0.0).from_global(f),
                         bmf=bx.MultiFab(ba).set_val(1.0).from_global(beta) if q["kind"] else None))
    alone = []
    for r in reqs:
        r["phi"].set_val(0.0)
        res = bx.mlmg_solve(r["phi"], r["rhs"], r["bmf"], precision=1, rel_tol=r["q"]["tol"])
        assert res.ok
        alone.append((r["phi"].to_global(), res))
        r["phi"].set_val(0.0)
    srv = bx.Server(reqs[0]["phi"].ctx, 256 << 20, max_problems=16, chunk=1, precision=1)
    got = {}
    # requests trickle in: two before every pump
    nxt = 0
    while len(got) < len(reqs):
        for _ in range(2):
            if nxt < len(reqs):
                r = reqs[nxt]
                srv.submit(nxt, r["phi"], r["rhs"], r["bmf"], r["q"]["tol"])
                nxt += 1
        for tag, res, _ in srv.pump():
            got[tag] = res
    assert not srv.rejected
    srv.close()
    mixed = 0
    for k, r in enumerate(reqs):
        u = r["phi"].to_global()
        assert got[k].ok and got[k].cycles == alone[k][1].cycles, k
        assert got[k].hist == alone[k][1].hist, k
        assert np.array_equal(u, alone[k][0]), k
        e = r["q"]["edge"]
        res = r["f"] - orc.apply_op((0, 0, 0), (e - 1,) * 3, (0, 0, 0), 1.0 / e, u, r["beta"])
        assert np.max(np.abs(res)) <= r["q"]["tol"] * np.max(np.abs(r["f"]))
        mixed += r["q"]["kind"]
    assert 0 < mixed < len(reqs)  # both coefficient kinds were served


def test_server_queues_when_full(bx):
    """A budget with room for one 64^3 problem: the rest wait in the queue
    and are admitted as earlier ones finish."""
    probs = []
    for s in range(3):
        ba = bx.BoxArray.chop((0, 0, 0), (63,) * 3, 32, bc=(bx.DIRICHLET0,) * 3)
        f = W.uniform_rhs((64, 64, 64), 90 + s)
        probs.append((bx.MultiFab(ba).set_val(0.0), bx.MultiFab(ba).set_val(0.0).from_global(f)))
    b = bx.Batch(probs[0][0].ctx, 64 << 20, 4)
    need = b.footprint(probs[0][0].ba)
    b.close()
    srv = bx.Server(probs[0][0].ctx, int(need * 1.5), max_problems=4, var_share=0.0)
    for k, (phi, rhs) in enumerate(probs):
        srv.submit(k, phi, rhs)
    order = []
    peak = 0
    while not srv.idle():
        out = srv.pump()
        peak = max(peak, srv.running() + len(out))
        order += [t for t, _, _ in out]
    assert order == [0, 1, 2] and peak == 1
    srv.close()
