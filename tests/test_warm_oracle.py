"""Pins of the oracle's warm start (Section 4.2: a guess for the primal, or
for the primal and dual variables).

* the initial point itself, read back with iter_max = 0, against its
  definition evaluated with the dense stacked rows of the QP: cold start
  (y = 0, pi = 0, lam = 1, t = max(Cy - d, 1)), primal guess (y kept, the rest
  as the cold start at that y) and primal-dual guess (kept, clamped below);
* a primal guess of zero is the cold start, bit for bit;
* a primal-dual guess at the solution exits at once with that point;
* warm-started solves reach the unique minimiser found by brute-force
  active-set enumeration and by the cold start.
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


def _tiny(seed):
    rng = np.random.default_rng(seed)
    return W.random_tiny(rng, int(rng.integers(2, 5)), nx_range=(1, 4), nu_range=(1, 3), ng_max=2), rng


@pytest.mark.parametrize("seed", range(6))
def test_initial_point_matches_definition(seed):
    qp, rng = _tiny(300 + seed)
    dq = DenseQp(qp)
    guess = random_interior_iterate(qp, rng, scale=0.7)
    if guess["lam_l"].size:
        guess["lam_l"][0] = 0.0   # below the clamps
        guess["t_u"][-1] = -0.5
    y = dq.y_from(guess["u"], guess["x"])
    for warm in (0, 1, 2):
        r = O.solve(qp, O.Arg.with_tol(1e-8, iter_max=0, warm_start=warm), guess=guess if warm else None)
        got_y = dq.y_from(r.sol["u"], r.sol["x"])
        if warm == 2:
            for k in KEYS:
                want = np.maximum(guess[k], 1e-16) if k.startswith(("lam", "t_")) else guess[k]
                assert np.array_equal(r.sol[k], want), (warm, k)
            continue
        y0 = y if warm == 1 else np.zeros_like(y)
        gy = dq.G @ y0
        assert np.array_equal(got_y, y0)
        assert np.all(r.sol["pi"] == 0.0)
        assert np.all(r.sol["lam_l"] == 1.0) and np.all(r.sol["lam_u"] == 1.0)
        assert np.allclose(r.sol["t_l"], np.maximum(gy - dq.lo, 1.0), rtol=0, atol=1e-14)
        assert np.allclose(r.sol["t_u"], np.maximum(dq.hi - gy, 1.0), rtol=0, atol=1e-14)


def test_zero_primal_guess_is_the_cold_start():
    qp = W.mass_spring_chain8(3)
    cold = O.solve(qp, O.Arg.with_tol(1e-8))
    zero = {k: np.zeros_like(v) for k, v in cold.sol.items()}
    warm = O.solve(qp, O.Arg.with_tol(1e-8, warm_start=1), guess=zero)
    assert warm.status == cold.status and warm.iters == cold.iters
    for k in KEYS:
        assert np.array_equal(warm.sol[k], cold.sol[k]), k


def test_guess_at_the_solution_exits_at_once():
    qp = W.mass_spring_chain4(1)
    ref = O.solve(qp, O.Arg.with_tol(1e-10))
    r = O.solve(qp, O.Arg.with_tol(1e-8, warm_start=2), guess=ref.sol)
    assert r.status == O.SUCCESS and r.iters == 0
    for k in KEYS:
        assert np.array_equal(r.sol[k], ref.sol[k]), k


@pytest.mark.parametrize("seed", range(6))
def test_warm_started_solve_reaches_brute_force_minimiser(seed):
    rng = np.random.default_rng(4000 + seed)
    while True:
        qp = W.random_tiny(rng, int(rng.integers(1, 3)), nx_range=(1, 3), nu_range=(1, 2), nb_frac=0.6, ng_max=1)
        dq = DenseQp(qp)
        nfree = int(np.sum(~np.isclose(dq.lo, dq.hi, rtol=0, atol=0)))
        if 1 <= nfree <= 8:
            break
    cands = dq.brute_force()
    if not cands:
        pytest.skip("random tiny QP infeasible")
    ystar = cands[0]
    guess = random_interior_iterate(qp, rng, scale=1.0)
    for warm in (1, 2):
        r = O.solve(qp, O.Arg.with_tol(1e-10, warm_start=warm), guess=guess)
        assert r.status == O.SUCCESS, (warm, r.status)
        assert rel(dq.y_from(r.sol["u"], r.sol["x"]), ystar) < 1e-7, warm
        assert O.kkt_res(qp, r.sol) <= 1e-10


def test_receding_horizon_warm_start_reaches_cold_minimiser():
    for i in range(4):
        qp = W.mass_spring_chain8(i)
        first = O.solve(qp, O.Arg.with_tol(1e-8))
        if first.status != O.SUCCESS:
            continue
        nxt, guess = W.receding_step(qp, first.sol)
        # tight tolerance: at KKT 1e-8 two points may differ by ~1e-5 (reading of the exit test)
        cold = O.solve(nxt, O.Arg.with_tol(1e-10))
        warm = O.solve(nxt, O.Arg.with_tol(1e-10, warm_start=2), guess=guess)
        assert cold.status == O.SUCCESS and warm.status == O.SUCCESS
        assert O.kkt_res(nxt, warm.sol) <= 1e-10
        for k in ("u", "x"):
            assert rel(warm.sol[k], cold.sol[k]) < 1e-6, (i, k)
