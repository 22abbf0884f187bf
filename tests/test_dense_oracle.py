"""Pins of the dense-QP oracle (full condensing, Section 3.5, and the dense
Cholesky IPM, Section 3.3) against what the definitions and the OCP oracle
fix, on the CPU:

* the condensed cost equals the sum of the stage costs along the trajectory
  the dynamics produce (up to the dropped constant), for random inputs and
  initial states;
* the condensed rows evaluate to the OCP rows (input and state boxes,
  general rows) along that trajectory;
* the dense IPM reaches the OCP oracle's minimiser (an independent solver:
  classical Riccati recursion on the uncondensed QP), and it fails where the
  OCP oracle fails;
* where both start from the same point, the dense IPM's iterates equal the
  OCP oracle's iteration by iteration: an independent implementation of the
  iteration control (initial point, centering rule, conditional corrector,
  step rule, clamps) pins the OCP oracle's, and a changed rule in it shows.
"""
import numpy as np
import pytest

from oracle import dense as D
from oracle import oracle as O
from paper_2003_02547_amd import workloads as W


def rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b))))


def tiny(i, **kw):
    rng = np.random.default_rng(700 + i)
    return W.random_tiny(rng, int(rng.integers(3, 9)), ng_max=2, **kw)


def cases():
    out = [W.mass_spring_chain4(1), W.mass_spring_chain8(3)] + [tiny(i) for i in range(8)]
    for i in range(3):
        out.append(W.random_tiny(np.random.default_rng(900 + i), 5, ng_max=2, x0_mode="free"))
        out.append(W.random_tiny(np.random.default_rng(950 + i), 5, ng_max=2, x0_mode="eliminated"))
    return out


def simulate(qp, v):
    """Inputs and states of the OCP QP from v = [u_0; ...; u_N; x_0], by
    stepping the dynamics stage by stage."""
    off = np.concatenate([[0], np.cumsum([qp.nu[n] for n in range(qp.N + 1)])]).astype(int)
    us = [v[off[n]:off[n] + qp.nu[n]] for n in range(qp.N + 1)]
    xs = [v[off[-1]:off[-1] + qp.nx[0]]]
    for n in range(qp.N):
        A = np.asarray(qp.A[n]).reshape(qp.nx[n + 1], qp.nx[n])
        B = np.asarray(qp.B[n]).reshape(qp.nx[n + 1], qp.nu[n])
        xs.append(A @ xs[n] + B @ us[n] + np.asarray(qp.b[n]))
    return us, xs


def stage_cost(qp, us, xs):
    c = 0.0
    for n in range(qp.N + 1):
        nu, nx = qp.nu[n], qp.nx[n]
        R = np.asarray(qp.R[n]).reshape(nu, nu)
        S = np.asarray(qp.S[n]).reshape(nu, nx)
        Q = np.asarray(qp.Q[n]).reshape(nx, nx)
        u, x = us[n], xs[n]
        c += 0.5 * u @ R @ u + u @ S @ x + 0.5 * x @ Q @ x + np.asarray(qp.r[n]) @ u + np.asarray(qp.q[n]) @ x
    return c


@pytest.mark.parametrize("k", range(6))
def test_condensed_cost_is_the_trajectory_cost(k):
    qp = cases()[k]
    dq = D.condense_dense(qp)
    rng = np.random.default_rng(k)
    v0 = np.zeros(dq.nv)
    base = stage_cost(qp, *simulate(qp, v0))
    for _ in range(3):
        v = rng.standard_normal(dq.nv)
        dense = 0.5 * v @ dq.H @ v + dq.g @ v
        assert abs(dense - (stage_cost(qp, *simulate(qp, v)) - base)) <= 1e-9 * max(1.0, abs(dense))


@pytest.mark.parametrize("k", range(6))
def test_condensed_rows_are_the_ocp_rows(k):
    qp = cases()[k]
    dq = D.condense_dense(qp)
    v = np.random.default_rng(10 + k).standard_normal(dq.nv)
    us, xs = simulate(qp, v)
    # box rows: every input box, then the state box of stage 0, by stage
    want_box, want_lo = [], []
    gen, glo = [], []
    for n in range(qp.N + 1):
        for j, i in enumerate(qp.idxbu[n]):
            want_box.append(us[n][i])
            want_lo.append(qp.lbu[n][j])
        if n == 0:
            for j, i in enumerate(qp.idxbx[n]):
                want_box.append(xs[0][i])
                want_lo.append(qp.lbx[0][j])
    box = v[dq.bidx]
    order = np.argsort(dq.bidx, kind="stable")
    assert np.allclose(np.sort(box), np.sort(want_box), atol=1e-12)
    assert np.allclose(np.sort(dq.blo), np.sort(want_lo))
    # general rows: state boxes of stages 1..N, then each stage's rows, by
    # stage; a row value minus its lower bound is the OCP row minus its bound
    for n in range(qp.N + 1):
        if n > 0:
            for j, i in enumerate(qp.idxbx[n]):
                gen.append(xs[n][i] - qp.lbx[n][j])
        Dn = np.asarray(qp.D[n]).reshape(-1, qp.nu[n]) if qp.nu[n] else np.zeros((len(qp.lg[n]), 0))
        Cn = np.asarray(qp.C[n]).reshape(Dn.shape[0], qp.nx[n])
        for j in range(Dn.shape[0]):
            gen.append(Dn[j] @ us[n] + Cn[j] @ xs[n] - qp.lg[n][j])
    assert order.size == box.size
    assert np.allclose(dq.C @ v - dq.glo, gen, atol=1e-10)


def test_dense_ipm_reaches_the_ocp_minimiser():
    for k, qp in enumerate(cases()):
        st, it, sol, norms = D.solve(qp, tol=1e-10)
        ref = O.solve(qp, O.Arg.with_tol(1e-10))
        assert (st == 0) == (ref.status == O.SUCCESS), (k, st, ref.status)
        if st != 0:
            continue
        assert np.max(norms) <= 1e-10
        assert abs(it - ref.iters) <= 1, (k, it, ref.iters)
        assert rel(sol["u"], ref.sol["u"]) <= 1e-7, (k, rel(sol["u"], ref.sol["u"]))
        assert rel(sol["x"], ref.sol["x"]) <= 1e-7, (k, rel(sol["x"], ref.sol["x"]))


def trajectory_cases():
    """QPs whose cold start satisfies the dynamics (b = 0, x0 as an
    equal-limit box): the OCP IPM and the dense IPM then start from the same
    point, and in exact arithmetic their Newton steps are the same step, so
    the two iterate sequences coincide up to rounding."""
    rng = lambda s: np.random.default_rng(np.random.SeedSequence([77, s]))
    return [W.mass_spring_chain4(1), W.mass_spring_chain8(3), W.random_stable(rng(1), 6, 3, 8),
            W.random_stable(rng(2), 5, 3, 6, ng=2)]


def test_iteration_control_pinned_by_the_dense_ipm():
    """The OCP oracle's iteration control (initial point, sigma = (mu_aff /
    mu)^3, the conditional corrector, the step rule, the clamps) against an
    independent implementation of the same rules on the dense QP: the
    primal iterates after k = 1..8 iterations agree to rounding."""
    for q in trajectory_cases():
        dq = D.condense_dense(q)
        for k in (1, 2, 3, 5, 8):
            _, _, v, *_ = D.solve_dense(dq, tol=1e-14, iter_max=k)
            sol = D.expand_dense(q, v)
            ref = O.solve(q, O.Arg.with_tol(1e-14, iter_max=k))
            assert rel(sol["u"], ref.sol["u"]) <= 1e-9, (k, rel(sol["u"], ref.sol["u"]))
            assert rel(sol["x"], ref.sol["x"]) <= 1e-9, (k, rel(sol["x"], ref.sol["x"]))


@pytest.mark.parametrize("change", [{"sigma_pow": 2.0}, {"corrector": False}, {"gamma": 0.9}])
def test_trajectory_comparison_notices_a_changed_rule(change):
    """The comparison above is sharp: a different centering power, a dropped
    corrector or another fraction to the boundary moves the dense iterates
    away from the OCP oracle's within a few iterations."""
    worst = 0.0
    for q in trajectory_cases():
        dq = D.condense_dense(q)
        _, _, v, *_ = D.solve_dense(dq, tol=1e-14, iter_max=3, **change)
        ref = O.solve(q, O.Arg.with_tol(1e-14, iter_max=3))
        worst = max(worst, rel(D.expand_dense(q, v)["u"], ref.sol["u"]))
    assert worst > 1e-6, worst
