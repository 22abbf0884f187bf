"""Pins of the oracle's soft constraints (Section 2.2: slack variables with
diagonal Hessians Zl, Zu, gradients zl, zu and lower bounds lls, lus,
eliminated row by row from the Newton system).

Each pin checks the oracle against something other than itself:
  * the residual function and the full Newton step of eq:alg:pdipm:delta on
    the generic QP in the augmented variables [y; s^l; s^u], built from the
    definition and solved by dense LU (no slack elimination);
  * the exact minimiser of tiny soft QPs by brute-force active sets on the
    same augmented QP;
  * a scalar problem with a closed-form solution, in both regimes of the
    linear penalty (slack active, and the exact-penalty regime where the
    soft solution is the hard one);
  * the exact-penalty property on a feasible mass-spring QP: with linear
    weights above the hard problem's multipliers, the soft minimiser is the
    hard one and the slacks vanish;
  * an infeasible hard instance becomes solvable, with a KKT point of the
    soft problem.
"""
import numpy as np
import pytest

from dense_ref import DenseSoftQp, random_interior_iterate_soft
from oracle import oracle as O
from paper_2003_02547_amd import workloads as W

ALL = ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u") + O.SOFT_NAMES


def _cmp(a, b, tol, what=""):
    for k in ALL:
        x, y = np.asarray(a[k]), np.asarray(b[k])
        assert x.shape == y.shape, (what, k, x.shape, y.shape)
        if x.size:
            err = np.max(np.abs(x - y)) / max(1.0, np.max(np.abs(y)))
            assert err <= tol, (what, k, err)


def soft_tiny(seed, N=None, **kw):
    """A tiny random QP with a random subset of its rows made soft."""
    rng = np.random.default_rng(seed)
    N = N if N is not None else int(rng.integers(1, 5))
    qp = W.random_tiny(rng, N, **kw)
    return W.soften_random(qp, rng), rng


@pytest.mark.parametrize("seed", range(12))
def test_soft_residual_matches_dense_definition(seed):
    qp, rng = soft_tiny(seed, ng_max=2)
    dq = DenseSoftQp(qp)
    it = random_interior_iterate_soft(qp, rng)
    parts, norms, mu = O.residuals(qp, it)
    rg, rb, rd, rm = dq.residual(it)
    ref = dq.split(rg, rd)
    for k in ("u", "x", "s_l", "s_u", "lam_l", "lam_u", "lam_sl", "lam_su"):
        assert np.allclose(parts[k], ref[k], atol=1e-12), k
    assert np.allclose(parts["pi"], rb, atol=1e-12)
    m, ns = dq.m, dq.ns
    assert np.allclose(np.concatenate([parts["t_l"], parts["t_u"], parts["t_sl"], parts["t_su"]]), rm, atol=1e-12)
    assert np.isclose(norms[0], np.max(np.abs(rg)), atol=1e-12)
    assert np.isclose(norms[2], np.max(np.abs(rd)), atol=1e-12)
    assert np.isclose(mu, np.sum(rm) / (2 * (m + ns)), atol=1e-12)


@pytest.mark.parametrize("seed", range(40))
def test_soft_newton_step_matches_dense_lu(seed):
    """The step with the slacks eliminated row by row == dense LU of the full
    Newton matrix of eq:alg:pdipm:delta over [y; s^l; s^u]."""
    mode = ["box", "free", "eliminated"][seed % 3]
    qp, rng = soft_tiny(seed, ng_max=2, x0_mode=mode)
    dq = DenseSoftQp(qp)
    it = random_interior_iterate_soft(qp, rng)
    tau = float(rng.uniform(0.0, 0.5))
    ref = dq.newton_step(it, tau)
    got = O.newton_step(qp, it, tau)
    _cmp(got, ref, 1e-9, f"seed {seed}")


@pytest.mark.parametrize("seed", range(10))
def test_soft_ipm_reaches_brute_force_minimiser(seed):
    rng = np.random.default_rng(2000 + seed)
    while True:
        s = int(rng.integers(1 << 30))
        qp, _ = soft_tiny(s, N=int(rng.integers(1, 3)), nx_range=(1, 3), nu_range=(1, 2), nb_frac=0.6, ng_max=1,
                          x0_mode=["box", "eliminated"][seed % 2])
        dq = DenseSoftQp(qp)
        nrows = dq.Cin.shape[0] - 2 * sum(1 for i in range(dq.m) if dq.lo[i] == dq.hi[i]
                                           and i not in set(dq.soft_rows))
        if 1 <= dq.ns and nrows <= 12:
            break
    cands = dq.brute_force()
    if not cands:
        pytest.skip("random tiny QP infeasible")
    ystar = cands[0]
    for y in cands[1:]:
        assert np.allclose(y, ystar, atol=1e-8)
    res = O.solve(qp, O.Arg.with_tol(1e-10))
    assert res.status == O.SUCCESS, res
    y = np.concatenate([dq.base.y_from(res.sol["u"], res.sol["x"]), res.sol["s_l"], res.sol["s_u"]])
    assert np.max(np.abs(y - ystar)) / max(1.0, np.max(np.abs(ystar))) < 1e-7


def _scalar(gamma, a=0.5, zeta=2.0):
    """x1 = x0 + u0 with x0 = 5 fixed, cost 1/2 u0^2 + 1/2 x0^2 + 1/2 a x1^2,
    soft box -100 <= x1 <= 0 (slack weights Z = zeta, z = gamma)."""
    one = np.ones((1, 1))
    qp = W.assemble(1, [1, 1], [1, 0], [one], [one], [np.zeros(1)], [one, a * one],
                    [np.zeros((1, 1)), np.zeros((0, 1))], [one, np.zeros((0, 0))], [np.zeros(1), np.zeros(1)],
                    [np.zeros(1), np.zeros(0)], boxx=[([0], [5.0], [5.0]), ([0], [-100.0], [0.0])])
    return W.soften(qp, lambda n, q: [0] if n == 1 else [], zeta, zeta, gamma, gamma)


@pytest.mark.parametrize("gamma", [0.0, 1.5, 4.0, 7.0, 20.0])
def test_scalar_closed_form(gamma):
    """Slack active: u = -(5 (a + zeta) + gamma) / (1 + a + zeta), x1 = s^u =
    (5 - gamma) / (1 + a + zeta).  For gamma >= 5 (the hard multiplier) the
    exact penalty holds: x1 = 0, s = 0, u = -5, lam_su = gamma - 5."""
    a, zeta = 0.5, 2.0
    res = O.solve(_scalar(gamma, a, zeta), O.Arg.with_tol(1e-12))
    assert res.status == O.SUCCESS
    x1 = max(0.0, (5.0 - gamma) / (1.0 + a + zeta))
    u = x1 - 5.0
    assert abs(res.sol["x"][1] - x1) < 1e-9
    assert abs(res.sol["u"][0] - u) < 1e-9
    assert abs(res.sol["s_u"][0] - x1) < 1e-9
    # with gamma = 0 the bound s^l >= 0 is weakly active (lam = t = 0 at the
    # solution), where an IPM at lam t <= 1e-12 stops ~sqrt(1e-12) away
    assert abs(res.sol["s_l"][0]) < (1e-5 if gamma == 0.0 else 1e-9)
    # the upper row's multiplier: zeta s^u + gamma while the slack is active,
    # the hard multiplier 5 (and lam_su = gamma - 5) once it is not
    lam = zeta * x1 + gamma if x1 > 0 else 5.0
    assert abs(res.sol["lam_u"][1] - lam) < 1e-8
    if x1 == 0.0:
        assert abs(res.sol["lam_su"][0] - (gamma - 5.0)) < 1e-8


def test_exact_penalty_recovers_the_hard_minimiser():
    qp = W.mass_spring_chain4(1)
    hard = O.solve(qp, O.Arg.with_tol(1e-12))
    assert hard.status == O.SUCCESS
    lam = np.max(np.abs(hard.sol["lam_l"] - hard.sol["lam_u"]))
    rows = lambda n, q: [k for k in range(q.nbu[n] + q.nbx[n] + q.ng[n]) if n > 0 or k < q.nbu[0]]
    sq = W.soften(qp, rows, 0.0, 0.0, 2.0 * lam + 1.0, 2.0 * lam + 1.0)
    soft = O.solve(sq, O.Arg.with_tol(1e-12))
    assert soft.status == O.SUCCESS
    for k in ("u", "x"):
        assert np.max(np.abs(soft.sol[k] - hard.sol[k])) < 1e-7, k
    assert np.max(np.abs(soft.sol["s_l"])) < 1e-8 and np.max(np.abs(soft.sol["s_u"])) < 1e-8


def test_soft_state_boxes_make_an_infeasible_instance_solvable():
    qp = W.mass_spring_chain8(222)
    assert O.solve(qp).status != O.SUCCESS
    sq = W.soften(qp, W.state_box_rows, 1.0, 1.0, 10.0, 10.0)
    res = O.solve(sq)
    assert res.status == O.SUCCESS
    assert O.kkt_res(sq, res.sol) <= 1e-8
    assert np.max(res.sol["s_l"]) > 1e-3 or np.max(res.sol["s_u"]) > 1e-3
    assert np.min(res.sol["s_l"]) > -1e-8 and np.min(res.sol["s_u"]) > -1e-8


def test_no_soft_rows_is_the_hard_problem():
    qp = W.mass_spring_chain4(3)
    hard = O.solve(qp)
    sq = W.soften(qp, lambda n, q: [], 1.0, 1.0, 1.0, 1.0)
    soft = O.solve(sq)
    assert soft.status == hard.status and soft.iters == hard.iters
    for k in ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u"):
        assert np.array_equal(soft.sol[k], hard.sol[k]), k


def test_soft_rejections():
    sq, _ = soft_tiny(5)
    with pytest.raises(ValueError):
        O.solve(sq, O.Arg(abs_form=1))
    bad = sq.copy()
    n = next(i for i in range(bad.N + 1) if len(bad.idxs[i]))
    bad.idxs[n] = np.concatenate([bad.idxs[n], bad.idxs[n][:1]])
    for k in ("Zl", "Zu", "zl", "zu", "lls", "lus"):
        getattr(bad, k)[n] = np.concatenate([getattr(bad, k)[n], getattr(bad, k)[n][:1]])
    with pytest.raises(ValueError):
        O.solve(bad)  # a row softened twice


# ---------------------------------------------------------------------------
# Warm start with slacks (Section 4.2): the primal guess includes s^l, s^u
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_soft_initial_point_matches_definition(seed):
    """iter_max = 0 returns the initial point: cold start (y' = 0), primal
    guess (y' = [y; s] kept, lam = 1, pi = 0, t = max(C'y' - d', 1) over every
    one-sided row of the augmented QP), primal-dual guess (kept, clamped)."""
    qp, rng = soft_tiny(400 + seed, ng_max=2)
    dq = DenseSoftQp(qp)
    guess = random_interior_iterate_soft(qp, rng, scale=0.7)
    if guess["lam_sl"].size:
        guess["lam_sl"][0] = 0.0   # below the clamps
        guess["t_su"][-1] = -0.5
    for warm in (0, 1, 2):
        r = O.solve(qp, O.Arg.with_tol(1e-8, iter_max=0, warm_start=warm), guess=guess if warm else None)
        if warm == 2:
            for k in ALL:
                want = np.maximum(guess[k], 1e-16) if k.startswith(("lam", "t_")) else guess[k]
                assert np.array_equal(r.sol[k], want), (warm, k)
            continue
        y0, _, _, _ = dq.stack(guess) if warm == 1 else (np.zeros(dq.nv), None, None, None)
        got = np.concatenate([dq.base.y_from(r.sol["u"], r.sol["x"]), r.sol["s_l"], r.sol["s_u"]])
        assert np.array_equal(got, y0), warm
        assert np.all(r.sol["pi"] == 0.0)
        lam = np.concatenate([r.sol[k] for k in ("lam_l", "lam_u", "lam_sl", "lam_su")])
        t = np.concatenate([r.sol[k] for k in ("t_l", "t_u", "t_sl", "t_su")])
        assert np.all(lam == 1.0)
        assert np.allclose(t, np.maximum(dq.Cin @ y0 - dq.d, 1.0), rtol=0, atol=1e-14), warm


def test_soft_primal_dual_guess_at_the_solution_exits_at_once():
    sq = W.mass_spring_chain8_soft(222)
    cold = O.solve(sq, O.Arg.with_tol(1e-10))
    assert cold.status == O.SUCCESS
    again = O.solve(sq, O.Arg.with_tol(1e-10, warm_start=2), guess=cold.sol)
    assert again.status == O.SUCCESS and again.iters == 0
    for k in ALL:
        assert np.array_equal(again.sol[k], np.maximum(cold.sol[k], 1e-16) if k.startswith(("lam", "t_"))
                              else cold.sol[k]), k


@pytest.mark.parametrize("warm", [1, 2])
def test_soft_warm_started_solves_reach_the_cold_minimiser(warm):
    for i in (0, 222, 350):
        sq = W.mass_spring_chain8_soft(i)
        cold = O.solve(sq, O.Arg.with_tol(1e-10))
        rng = np.random.default_rng(i)
        guess = {k: v + 0.05 * rng.standard_normal(v.shape) for k, v in cold.sol.items()}
        for k in guess:
            if k.startswith(("lam", "t_")):
                guess[k] = np.maximum(guess[k], 1.0)
        ws = O.solve(sq, O.Arg.with_tol(1e-10, warm_start=warm), guess=guess)
        assert ws.status == O.SUCCESS, (i, warm)
        y = np.concatenate([ws.sol[k] for k in ("u", "x", "s_l", "s_u")])
        yc = np.concatenate([cold.sol[k] for k in ("u", "x", "s_l", "s_u")])
        # instance 0 has a weakly active input bound (lam and t both ~0 at
        # the solution): there two KKT points at lam t <= 1e-10 can differ
        # by ~sqrt(1e-10) in that input
        assert np.max(np.abs(y - yc)) / max(1.0, np.max(np.abs(yc))) < 1e-5, (i, warm)
        assert O.kkt_res(sq, ws.sol) <= 1e-10
