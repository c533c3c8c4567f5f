"""GPU parity of the nodal Poisson solve against the oracle's, through the
C ABI (bxmg_nodal_solve).

Bar: fixed-cycle iterates equal the oracle's to 1e-12 relative (the stages
take the oracle's operation order; the bottom CG sums in another order),
the residual history matches to 1e-6 while above 1e-6 ||f||, a full solve
meets 1e-10 by the oracle's operator and agrees with the oracle's solution
within the error bound; closed-form eigenvector solutions; periodic copies
equal their nodes; argument errors.
"""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bx():
    import paper_2403_12179_amd as bx
    return bx


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).transpose(2, 1, 0))).cuda()


def host(t):
    return np.asfortranarray(t.cpu().numpy().transpose(2, 1, 0))


def nodes(n):
    return tuple(x + 1 for x in n)


def unknown_mask(n, per):
    m = np.ones(nodes(n), bool)
    for d in range(3):
        for c in ([n[d]] if per[d] else [0, n[d]]):
            sl = [slice(None)] * 3
            sl[d] = c
            m[tuple(sl)] = False
    return m


CASES = [((64, 64, 64), (0, 0, 0)), ((32, 48, 32), (1, 1, 1)), ((48, 32, 64), (1, 0, 0)), ((40, 40, 40), (0, 1, 0))]


@pytest.mark.parametrize("n,per", CASES)
def test_nodal_matches_oracle(bx, orc, n, per):
    bc = tuple(bx.PERIODIC if p else bx.DIRICHLET0 for p in per)
    ba = bx.BoxArray.chop((0, 0, 0), tuple(x - 1 for x in n), 32, bc=bc)
    m = unknown_mask(n, per)
    f = np.asfortranarray(W.uniform_rhs(nodes(n), 61))
    if per == (1, 1, 1):
        f = np.asfortranarray(f - f[m].mean())
    h = 1.0 / n[0]
    phi, rhs = dev(np.zeros(nodes(n))), dev(f)
    res = bx.nodal_solve(ba, phi, rhs, fixed_cycles=3)
    uo, io = orc.nodal_solve(n, per, f, fixed_cycles=3)
    assert res.cycles == 3 and io["cycles"] == 3 and res.levels == io["levels"]
    u = host(phi)
    assert np.max(np.abs(u - uo)) <= 1e-12 * np.max(np.abs(uo))
    phi.zero_()
    res = bx.nodal_solve(ba, phi, rhs)
    assert res.ok, res
    u = host(phi)
    r = np.where(m, f - orc.nodal_apply(n, per, h, u), 0.0)
    assert np.max(np.abs(r)) <= 1e-10 * np.max(np.abs(f[m]))
    uo, io = orc.nodal_solve(n, per, f)
    assert abs(res.cycles - io["cycles"]) <= 1
    for k in range(min(len(res.hist), len(io["hist"]))):
        a, b = res.hist[k], io["hist"][k]
        if b >= 1e-6:
            assert abs(a - b) <= 1e-6 * b, (k, a, b)
    assert np.max(np.abs(u - uo)) <= 0.405 * max(n) ** 2 * 2e-10 * np.max(np.abs(uo))
    for d in range(3):  # periodic copies equal their nodes
        if per[d]:
            a = np.take(u, 0, axis=d)
            b = np.take(u, n[d], axis=d)
            assert np.array_equal(a, b)


@pytest.mark.parametrize("per", [(0, 0, 0), (1, 1, 1)])
def test_nodal_sine_closed_form(bx, per):
    m = 32
    n = (m, m, m)
    h = 1.0 / m
    k = 2 * np.pi if per[0] else np.pi
    s1 = np.sin(k * np.arange(m + 1) * h)
    s = np.einsum("i,j,k->ijk", s1, s1, s1)
    lam = 12.0 * np.sin(k * h / 2) ** 2 / h ** 2
    bc = tuple(bx.PERIODIC if p else bx.DIRICHLET0 for p in per)
    ba = bx.BoxArray.chop((0, 0, 0), (m - 1,) * 3, 16, bc=bc)
    phi, rhs = dev(np.zeros(nodes(n))), dev(s)
    res = bx.nodal_solve(ba, phi, rhs)
    assert res.ok
    assert np.max(np.abs(host(phi) + s / lam)) <= 1e-9 / lam


def test_nodal_arguments(bx):
    ba = bx.BoxArray.chop((0, 0, 0), (15, 15, 15), 16)
    phi, rhs = dev(np.zeros((17, 17, 17))), dev(np.zeros((17, 17, 17)))
    lib = bx.lib()
    info = bx._lib.SolveInfo()
    for kw in (dict(precision=1), dict(krylov=1), dict(alpha=1.0)):
        p = bx.solve_params(**kw)
        assert lib.bxmg_nodal_solve(bx.default_context()._h, C.byref(p), ba._h, C.c_void_p(phi.data_ptr()),
                                    C.c_void_p(rhs.data_ptr()), C.byref(info)) == -1
    res = bx.nodal_solve(ba, phi, rhs)  # f = 0: u = 0
    assert res.ok and res.cycles == 0
    bad = np.zeros((17, 17, 17))
    bad[4, 5, 6] = np.nan
    res = bx.nodal_solve(ba, phi, dev(bad))
    assert res.status == -5
    with pytest.raises(ValueError):
        bx.nodal_solve(ba, dev(np.zeros((17, 17, 16))), rhs)
