"""Pins of the oracle's absolute formulation (Section 3.2, eq:alg:pdipm:abs
and eq:alg:pdipm:step; mode speed_abs of Section 4.2).

* the step equals the difference between the dense solution of
  eq:alg:pdipm:abs, written out from the stacked QP (right-hand side
  -[g; b; d; -Lam T e - tau e]), and the current iterate;
* it equals the delta-formulation step (the same Newton step in exact
  arithmetic) at iterates away from the solution;
* the loop: the first iterations follow the delta formulation's iterates,
  and the exit is on the duality measure alone (residuals only before
  returning).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_02547_amd import workloads as W
from dense_ref import DenseQp, random_interior_iterate

KEYS = ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u")


def rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b))))


@pytest.mark.parametrize("seed", range(8))
def test_abs_step_is_dense_solution_minus_iterate(seed):
    rng = np.random.default_rng(500 + seed)
    qp = W.random_tiny(rng, int(rng.integers(1, 5)), nx_range=(1, 4), nu_range=(0, 3), ng_max=2,
                       x0_mode=["box", "free", "eliminated"][seed % 3])
    it = random_interior_iterate(qp, rng, scale=0.6)
    tau = float(rng.uniform(0.0, 0.3))
    dq = DenseQp(qp)
    y, pi, lam, t = dq.stack(it)
    K = dq.kkt_matrix(it)
    rhs = -np.concatenate([dq.g, dq.beq, dq.d, -lam * t - tau])
    full = np.linalg.solve(K, rhs)
    cur = np.concatenate([y, pi, lam, t])
    want = dq.unstack_step(full - cur)
    got = O.newton_step(qp, it, tau, abs_form=True)
    delta = O.newton_step(qp, it, tau)
    for k in KEYS:
        assert rel(got[k], want[k]) < 1e-9, (seed, k, rel(got[k], want[k]))
        assert rel(got[k], delta[k]) < 1e-9, (seed, k)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_first_iterations_follow_the_delta_formulation(k):
    qp = W.mass_spring_chain4(1)
    d = O.solve(qp, O.Arg.with_tol(1e-8, iter_max=k))
    a = O.solve(qp, O.Arg.with_tol(1e-8, iter_max=k, abs_form=1))
    assert d.iters == a.iters == k
    for key in KEYS:
        assert rel(a.sol[key], d.sol[key]) < 1e-9, (k, key)


@pytest.mark.parametrize("tol", [1e-4, 1e-6, 1e-8])
def test_exit_on_the_duality_measure(tol):
    qp = W.mass_spring_chain8(5)
    r = O.solve(qp, O.Arg.with_tol(tol, abs_form=1))
    assert r.status == O.SUCCESS and r.mu <= tol
    before = O.solve(qp, O.Arg.with_tol(tol, abs_form=1, iter_max=r.iters - 1))
    assert before.status == O.MAX_ITER and before.mu > tol
    # the residual norms are those of the returned point
    _, norms, mu = O.residuals(qp, r.sol)
    assert np.allclose(norms, r.res, rtol=1e-12, atol=1e-300) and abs(mu - r.mu) <= 1e-12 * max(1.0, mu)


@pytest.mark.parametrize("seed", range(4))
def test_abs_solve_reaches_the_minimiser_loosely(seed):
    """Cancellation limits the accuracy of the absolute formulation near the
    solution (Section 3.2); at a moderate tolerance it still lands near the
    brute-force minimiser."""
    rng = np.random.default_rng(6000 + seed)
    while True:
        qp = W.random_tiny(rng, int(rng.integers(1, 3)), nx_range=(1, 3), nu_range=(1, 2), nb_frac=0.6, ng_max=1)
        dq = DenseQp(qp)
        nfree = int(np.sum(~np.isclose(dq.lo, dq.hi, rtol=0, atol=0)))
        if 1 <= nfree <= 8:
            break
    cands = dq.brute_force()
    if not cands:
        pytest.skip("random tiny QP infeasible")
    r = O.solve(qp, O.Arg.with_tol(1e-6, abs_form=1))
    assert r.status == O.SUCCESS
    assert rel(dq.y_from(r.sol["u"], r.sol["x"]), cands[0]) < 1e-3
