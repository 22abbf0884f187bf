"""Pins of the oracle's partial condensing (Section 3.5) against facts it does
not compute itself:

* with one stage per block the condensed QP is the original QP;
* at any point (u_bar, x_bar) the condensed cost, constraint rows and block-end
  state equal the original ones along the trajectory obtained by stepping the
  dynamics forward (the oracle instead solves the block's stacked dynamics);
* the condensed QP has the same minimiser as the original (Section 3.5: the
  eliminated states are determined by the inputs and the block-start state),
  checked against brute-force active-set enumeration and against the oracle
  IPM on the original QP, and the expanded primal-dual point satisfies the
  original KKT conditions eq:alg:pdipm:kkt.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import pcond as PC
from paper_2003_02547_amd import workloads as W
from dense_ref import DenseQp

FIELDS = ("A", "B", "b", "Q", "S", "R", "q", "r", "idxbu", "lbu", "ubu", "idxbx", "lbx", "ubx", "D", "C", "lg", "ug")


def rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b))))


@pytest.mark.parametrize("N,N2", [(10, 3), (30, 5), (30, 15), (7, 7), (5, 9), (12, 1), (1, 1)])
def test_block_starts(N, N2):
    s = PC.block_starts(N, N2)
    L = np.diff(s)
    assert s[0] == 0 and s[-1] == N and len(s) == min(N, N2) + 1
    assert L.min() >= 1 and L.max() - L.min() <= 1
    assert np.all(np.diff(L) <= 0)  # longer blocks first


def test_one_stage_per_block_is_identity():
    rng = np.random.default_rng(5)
    qp = W.random_tiny(rng, 5, nx_range=(1, 4), nu_range=(0, 3), ng_max=2)
    cq = PC.condense(qp, qp.N)
    assert cq.N == qp.N and list(cq.nx) == list(qp.nx) and list(cq.nu) == list(qp.nu)
    for f in FIELDS:
        for n, (a, b) in enumerate(zip(getattr(cq, f), getattr(qp, f))):
            assert np.array_equal(np.asarray(a), np.asarray(b)), (f, n)


def _simulate_block(qp, s0, s1, ub, xb):
    """Trajectory of one block by stepping the dynamics forward."""
    u, x = [], [xb]
    o = 0
    for n in range(s0, s1):
        u.append(ub[o:o + qp.nu[n]])
        o += qp.nu[n]
        if n < qp.N:
            x.append(qp.A[n] @ x[-1] + qp.B[n] @ u[-1] + qp.b[n])
    return u, x


def _stage_cost(qp, n, u, x):
    z = np.concatenate([u, x])
    H = np.block([[qp.R[n], qp.S[n]], [np.asarray(qp.S[n]).T, qp.Q[n]]]) if qp.nu[n] and qp.nx[n] else \
        (np.asarray(qp.R[n]) if qp.nu[n] else np.asarray(qp.Q[n]))
    return 0.5 * z @ H @ z + np.concatenate([qp.r[n], qp.q[n]]) @ z


@pytest.mark.parametrize("seed,N,N2", [(0, 6, 2), (1, 7, 3), (2, 5, 1), (3, 9, 4)])
def test_condensed_data_matches_forward_simulation(seed, N, N2):
    rng = np.random.default_rng(100 + seed)
    qp = W.random_tiny(rng, N, nx_range=(1, 4), nu_range=(1, 3), nb_frac=0.6, ng_max=2)
    cq = PC.condense(qp, N2)
    s = PC.block_starts(N, N2)
    blocks = [(s[b], s[b + 1]) for b in range(len(s) - 1)] + [(N, N + 1)]
    for b, (s0, s1) in enumerate(blocks):
        nU, nxs = cq.nu[b], cq.nx[b]
        diffs = []
        for _ in range(3):
            ub, xb = rng.standard_normal(nU), rng.standard_normal(nxs)
            u, x = _simulate_block(qp, s0, s1, ub, xb)
            orig = sum(_stage_cost(qp, n, u[k], x[k]) for k, n in enumerate(range(s0, s1)))
            zb = np.concatenate([ub, xb])
            Hb = np.block([[cq.R[b], cq.S[b]], [cq.S[b].T, cq.Q[b]]])
            cond = 0.5 * zb @ Hb @ zb + np.concatenate([cq.r[b], cq.q[b]]) @ zb
            diffs.append(orig - cond)  # equal up to the constant dropped by condensing
            if b < len(s) - 1:
                assert rel(cq.A[b] @ xb + cq.B[b] @ ub + cq.b[b], x[-1]) < 1e-12
            # constraint rows: value minus bound, original vs condensed
            want_lo, want_hi, got_lo, got_hi = [], [], [], []
            for k, n in enumerate(range(s0, s1)):
                if k >= 1:
                    for j in np.argsort(qp.idxbx[n], kind="stable"):
                        i = qp.idxbx[n][j]
                        want_lo.append(x[k][i] - qp.lbx[n][j]); want_hi.append(qp.ubx[n][j] - x[k][i])
                gv = np.asarray(qp.D[n]) @ u[k] + np.asarray(qp.C[n]) @ x[k]
                want_lo += list(gv - qp.lg[n]); want_hi += list(qp.ug[n] - gv)
            cg = cq.D[b] @ ub + cq.C[b] @ xb
            got_lo, got_hi = cg - cq.lg[b], cq.ug[b] - cg
            assert rel(got_lo, want_lo) < 1e-12 and rel(got_hi, want_hi) < 1e-12
            # boxes: inputs at their offsets, the first state of the block
            o = np.concatenate([[0], np.cumsum([qp.nu[n] for n in range(s0, s1)])])
            expect_u = sorted(o[k] + i for k, n in enumerate(range(s0, s1)) for i in qp.idxbu[n])
            assert list(cq.idxbu[b]) == expect_u
            assert sorted(cq.idxbx[b]) == sorted(qp.idxbx[s0])
        assert max(diffs) - min(diffs) < 1e-10 * max(1.0, abs(diffs[0]))


@pytest.mark.parametrize("seed", range(6))
def test_condensed_minimiser_is_the_brute_force_one(seed):
    rng = np.random.default_rng(2000 + seed)
    while True:
        qp = W.random_tiny(rng, 2, nx_range=(1, 2), nu_range=(1, 2), nb_frac=0.6, ng_max=1)
        dq = DenseQp(qp)
        nfree = int(np.sum(~np.isclose(dq.lo, dq.hi, rtol=0, atol=0)))
        if 1 <= nfree <= 8:
            break
    cands = dq.brute_force()
    if not cands:
        pytest.skip("random tiny QP infeasible")
    ystar = cands[0]
    cq = PC.condense(qp, 1)
    res = O.solve(cq, O.Arg.with_tol(1e-10))
    assert res.status == O.SUCCESS, res
    sol = PC.expand(qp, 1, res.sol)
    y = dq.y_from(sol["u"], sol["x"])
    assert rel(y, ystar) < 1e-7
    assert O.kkt_res(qp, sol) < 1e-8


@pytest.mark.parametrize("case", ["tiny6_2", "tiny8_3", "chain4_2", "chain4_5", "chain8_5", "uneven_4"])
def test_expanded_solution_matches_original_solve(case):
    if case.startswith("tiny"):
        N, N2 = int(case[4]), int(case[-1])
        rng = np.random.default_rng(N * 10 + N2)
        for _ in range(20):  # first feasible draw of the stream
            qp = W.random_tiny(rng, N, nx_range=(2, 4), nu_range=(1, 3), ng_max=1)
            if O.solve(qp, O.Arg.with_tol(1e-10)).status == O.SUCCESS:
                break
    elif case.startswith("chain4"):
        qp, N2 = W.mass_spring_chain4(1), int(case[-1])
    elif case.startswith("chain8"):
        qp, N2 = W.mass_spring_chain8(0), int(case[-1])
    else:
        qp, N2 = W.random_uneven(3), int(case[-1])
    ref = O.solve(qp, O.Arg.with_tol(1e-10))
    assert ref.status == O.SUCCESS
    cq = PC.condense(qp, N2)
    assert cq.N == min(N2, qp.N)
    res = O.solve(cq, O.Arg.with_tol(1e-10))
    assert res.status == O.SUCCESS
    sol = PC.expand(qp, N2, res.sol)
    for k in ("u", "x"):
        assert rel(sol[k], ref.sol[k]) < 1e-6, k
    assert O.kkt_res(qp, sol) < 1e-8
    # same number of two-sided constraints (mu is comparable)
    nc = lambda q: sum(len(a) + len(b) + np.asarray(d).shape[0] for a, b, d in zip(q.idxbu, q.idxbx, q.D))
    assert nc(cq) == nc(qp)
