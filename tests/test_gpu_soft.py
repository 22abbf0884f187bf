"""GPU parity of soft constraints (Section 2.2) against the oracle: the soft
builds of the one-wave kernel and of the block kernel, called through the
C-ABI.

* the Newton step at random interior iterates (slack blocks included) on
  tiny random soft QPs: every block element by element, 1e-9;
* full solves of tiny and small random soft QPs (random subsets of box and
  general rows softened, random weights and slack bounds): same status,
  iteration counts within one at tolerance 1e-6, primal (u, x, s^l, s^u) within 1e-6 and the
  oracle's KKT residual of the returned point (slack rows included) within
  the tolerance;
* the 8-mass batch of 1024 with soft position boxes (the instances whose
  hard boxes are infeasible included): all solved, sampled against the
  oracle;
* the uneven batch with its first x0 draws and soft state boxes, stage
  blocks up to 64 and above (global-memory mode), sampled;
* a batch mixing QPs with and without slacks, and edge cases: a stage with
  every row soft, soft general rows, soft rows with equal limits, a QP whose
  slack count is zero at every stage inside a soft batch.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2003_02547_amd import binding as B  # noqa: E402
from paper_2003_02547_amd import workloads as W  # noqa: E402
from dense_ref import random_interior_iterate_soft  # noqa: E402

ALL = ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u") + O.SOFT_NAMES


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    B.lib()


def soft_tiny(seed, frac=0.6, **kw):
    rng = np.random.default_rng(seed)
    N = kw.pop("N", None) or int(rng.integers(1, 9))
    qp = W.random_tiny(rng, N, **kw)
    return W.soften_random(qp, rng, frac), rng


def primal(sol):
    return np.concatenate([sol["u"], sol["x"], sol.get("s_l", []), sol.get("s_u", [])])


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b)))) if b.size else 0.0


@pytest.fixture
def wave_bound():
    L = B.lib()
    old = L.oqp_get_wave_max()
    yield L
    L.oqp_set_wave_max(old)


@pytest.mark.parametrize("wmax", [24, 0])
def test_soft_newton_step_matches_oracle(wmax, wave_bound):
    """wmax 24: the one-wave kernel's soft build; 0: every instance on the
    block kernel's soft build."""
    wave_bound.oqp_set_wave_max(wmax)
    qps, its = [], []
    for seed in range(48):
        qp, rng = soft_tiny(seed, nx_range=(1, 6), nu_range=(0, 4), ng_max=3,
                            x0_mode=["box", "free", "eliminated"][seed % 3])
        qps.append(qp)
        its.append(random_interior_iterate_soft(qp, rng))
    say(f"soft Newton step x48 vs oracle, wave bound {wmax}")
    b = B.Batch(qps, B.default_arg()).load()
    groups = {b.variant(i)[0] for i in range(len(qps))}
    nv = B.lib().oqp_variant_count()
    assert (max(groups) >= nv) if wmax == 0 else (min(groups) < nv)
    for i, it in enumerate(its):
        b.set_iterate(i, it)
    b.newton(0.3).fetch().sync()
    for i, (qp, it) in enumerate(zip(qps, its)):
        got = b.step(i)
        ref = O.newton_step(qp, it, 0.3)
        for k in ALL:
            if k in ref and ref[k].size:
                assert rel(got[k], ref[k]) <= 1e-9, (i, k, rel(got[k], ref[k]))


@pytest.mark.parametrize("sizes", [dict(nx_range=(1, 5), nu_range=(0, 3), ng_max=2, frac=0.6),
                                   dict(nx_range=(8, 20), nu_range=(2, 8), ng_max=6, frac=1.0),
                                   dict(nx_range=(30, 40), nu_range=(10, 20), ng_max=8, frac=1.0)])
def test_soft_solves_match_oracle(sizes):
    qps = [soft_tiny(100 + s, **sizes)[0] for s in range(24)]
    say(f"soft solves x24 {sizes} vs oracle")
    res = B.solve(qps, B.default_arg())
    # the trajectory at 1e-6, away from the rounding floor: on the larger
    # random draws the stationarity residual stalls just under 1e-8, where
    # the square-root and the classical factorization, rounding differently,
    # cross the tolerance a few iterations apart
    res6 = B.solve(qps, B.default_arg(tol_stat=1e-6, tol_eq=1e-6, tol_ineq=1e-6, tol_comp=1e-6))
    nok = 0
    for i, (qp, r, r6) in enumerate(zip(qps, res, res6)):
        ref = O.solve(qp)
        if ref.status != O.SUCCESS:
            # an infeasible draw (hard rows left): both fail, the failure
            # mode at the breakdown may differ (MIN_STEP / NaN)
            assert r.status != B.SUCCESS, (i, r.status, ref.status)
            continue
        nok += 1
        assert r.status == B.SUCCESS, (i, r.status, r.iters, ref.iters)
        assert O.kkt_res(qp, r.sol) <= 1e-8 * 1.01, (i, O.kkt_res(qp, r.sol))
        assert rel(primal(r.sol), primal(ref.sol)) <= 1e-6, (i, rel(primal(r.sol), primal(ref.sol)))
        ref6 = O.solve(qp, O.Arg.with_tol(1e-6))
        assert r6.status == ref6.status == O.SUCCESS, i
        assert abs(r6.iters - ref6.iters) <= 1, (i, r6.iters, ref6.iters)
    assert nok >= 18


def test_chain8_soft_full_batch_sampled():
    qps = [W.mass_spring_chain8_soft(i) for i in range(1024)]
    say("8-mass x1024 with soft position boxes, sampled vs oracle")
    res = B.solve(qps, B.default_arg())
    assert all(r.status == B.SUCCESS for r in res)
    for i in list(range(0, 1024, 64)) + [222, 350]:
        ref = O.solve(qps[i])
        assert ref.status == O.SUCCESS
        assert O.kkt_res(qps[i], res[i].sol) <= 1e-8 * 1.01, i
        assert rel(primal(res[i].sol), primal(ref.sol)) <= 1e-6, (i, rel(primal(res[i].sol), primal(ref.sol)))
    # the hard instance 222 is infeasible: its soft solution uses the slacks
    assert max(res[222].sol["s_l"].max(), res[222].sol["s_u"].max()) > 1e-3


def test_uneven_soft_sampled():
    qps = [W.random_uneven_soft(i) for i in range(512)]
    say("uneven x512 with first x0 draws and soft state boxes, sampled vs oracle")
    b = B.Batch(qps, B.default_arg(), streams=3).load().solve().fetch().sync()
    res = b.results()
    assert sum(r.status == B.SUCCESS for r in res) == len(qps)
    picks = list(range(0, 512, 32)) + [7, 18, 19]
    for i in picks:
        ref = O.solve(qps[i])
        assert ref.status == O.SUCCESS
        assert O.kkt_res(qps[i], res[i].sol) <= 1e-8 * 1.01, i
        assert rel(primal(res[i].sol), primal(ref.sol)) <= 1e-6, i
    # the batch covers the LDS and the global-memory modes
    groups = {b.variant(i)[0] for i in range(len(qps))}
    assert len(groups) >= 2


def test_large_stage_soft_global_memory_mode():
    qps = [W.soften(W.random_large_stage(i), W.state_box_rows, W.SOFT_Z, W.SOFT_Z, W.SOFT_z, W.SOFT_z)
           for i in range(8)]
    say("large-stage x8 (nx 128, nu 32, ng 32) with soft state boxes vs oracle, tolerance 1e-6")
    # the metric's tolerance, as for the hard large-stage batch: at 1e-8 the
    # oracle's stationarity residual stalls at ~1e-7 on these stages as well
    tol = dict(tol_stat=1e-6, tol_eq=1e-6, tol_ineq=1e-6, tol_comp=1e-6)
    res = B.solve(qps, B.default_arg(**tol))
    assert all(r.status == B.SUCCESS for r in res)
    for i in (0, 5):
        ref = O.solve(qps[i], O.Arg.with_tol(1e-6))
        assert ref.status == O.SUCCESS
        assert abs(res[i].iters - ref.iters) <= 1, (i, res[i].iters, ref.iters)
        assert O.kkt_res(qps[i], res[i].sol) <= 1e-6 * 1.01, i
        assert rel(primal(res[i].sol), primal(ref.sol)) <= 1e-6, i


def _edge_cases():
    rng = np.random.default_rng(77)
    out = []
    # every row of every stage soft (stage 0's x0 rows included)
    qp = W.random_tiny(rng, 4, nx_range=(2, 4), nu_range=(1, 3), ng_max=2)
    out.append(W.soften(qp, lambda n, q: range(q.nbu[n] + q.nbx[n] + q.ng[n]), 2.0, 2.0, 1.0, 1.0))
    # soft general rows and state boxes, hard input boxes
    qp = W.random_tiny(rng, 5, nx_range=(2, 4), nu_range=(1, 3), ng_max=3)
    out.append(W.soften(qp, lambda n, q: range(q.nbu[n] if n else q.nbu[n] + q.nbx[n], q.nbu[n] + q.nbx[n] + q.ng[n]),
                        0.5, 0.5, 3.0, 3.0))
    # soft rows with equal limits (an equality made soft) and no linear weight
    qp = W.random_tiny(rng, 3, nx_range=(2, 3), nu_range=(1, 2), ng_max=0)
    for n in range(1, 4):
        if len(qp.idxbx[n]):
            qp.lbx[n][0] = qp.ubx[n][0] = 0.1
    out.append(W.soften(qp, W.state_box_rows, 1.0, 1.0, 0.0, 0.0))
    # no slacks at any stage
    out.append(W.soften(W.mass_spring_chain4(7), lambda n, q: [], 1.0, 1.0, 1.0, 1.0))
    return out


def test_soft_edge_cases_and_mixed_batch():
    edge = _edge_cases()
    hard = [W.mass_spring_chain4(s) for s in range(1, 5)]
    qps = edge + hard
    say("soft edge cases + QPs without slacks in one soft batch vs oracle")
    res = B.solve(qps, B.default_arg())
    for i, (qp, r) in enumerate(zip(qps, res)):
        ref = O.solve(qp)
        assert ref.status == O.SUCCESS, i
        assert r.status == B.SUCCESS, (i, r.status)
        assert O.kkt_res(qp, r.sol) <= 1e-8 * 1.01, (i, O.kkt_res(qp, r.sol))
        assert rel(primal(r.sol), primal(ref.sol)) <= 1e-6, i
    # the QPs without slacks solve as they do in a batch of their own
    alone = B.solve(hard, B.default_arg())
    for a, r in zip(alone, res[len(edge):]):
        assert a.status == r.status == B.SUCCESS
        assert rel(primal(r.sol), primal(a.sol)) <= 1e-6


def test_soft_batch_rejects_other_modes():
    qp = W.mass_spring_chain8_soft(0)
    for kw in (dict(mode=B.MODE_MIXED), dict(mode=B.MODE_ABS), dict(mode=B.MODE_ROBUST), dict(mode=B.MODE_BALANCE),
               dict(cond_N=5)):
        mode = kw.pop("mode", B.MODE_F64)
        with pytest.raises(B.OqpError):
            B.Batch([qp], B.default_arg(mode, **kw))


# ---------------------------------------------------------------------------
# warm start with slacks (Section 4.2)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("wmax", [24, 0])
def test_soft_initial_point_parity(wmax, wave_bound):
    """iter_max = 0: the cold start, a primal guess (slacks included) and a
    primal-dual guess equal the oracle's initial points, one-wave (24) and
    block (0) kernels."""
    wave_bound.oqp_set_wave_max(wmax)
    qps, guesses = [], []
    for seed in range(8):
        qp, rng = soft_tiny(500 + seed, nx_range=(1, 5), nu_range=(1, 3), ng_max=2)
        g = random_interior_iterate_soft(qp, rng, scale=0.7)
        if g["lam_sl"].size:
            g["lam_sl"][0] = 0.0   # below the clamps
            g["t_su"][-1] = -0.5
        qps.append(qp)
        guesses.append(g)
    say(f"soft warm start initial point parity, wave bound {wmax}")
    for warm in (0, 1, 2):
        b = B.Batch(qps, B.default_arg(iter_max=0, warm_start=warm)).load()
        for i in range(len(qps)):
            if warm:
                b.set_iterate(i, guesses[i])
        b.solve().fetch().sync()
        for i, q in enumerate(qps):
            ref = O.solve(q, O.Arg.with_tol(1e-8, iter_max=0, warm_start=warm), guess=guesses[i] if warm else None)
            got = b.solution(i)
            for k in ALL:
                assert rel(got[k], ref.sol[k]) <= 1e-14, (warm, i, k, rel(got[k], ref.sol[k]))


def test_soft_receding_horizon_warm_solves_follow_the_oracle():
    """The next receding-horizon problem of each solved soft 8-mass instance
    (x_0 <- x_1), warm-started from the shifted solution with its slacks:
    the oracle's warm-started iterations, the KKT tolerance, fewer
    iterations than cold starts."""
    qps = [W.mass_spring_chain8_soft(i) for i in range(64)] + [W.mass_spring_chain8_soft(222)]
    say("soft receding horizon, warm (primal-dual guess) vs oracle")
    first = B.solve(qps, B.default_arg())
    assert all(r.status == B.SUCCESS for r in first)
    nxt, guesses = zip(*[W.receding_step(q, r.sol) for q, r in zip(qps, first)])
    b = B.Batch(list(nxt), B.default_arg(warm_start=2)).load()
    for i, g in enumerate(guesses):
        b.set_iterate(i, g)
    b.solve().fetch().sync()
    warm = b.results()
    cold = B.solve(list(nxt), B.default_arg())
    assert sum(r.iters for r in warm) < sum(r.iters for r in cold)
    for i in list(range(0, 64, 9)) + [64]:
        ref = O.solve(nxt[i], O.Arg.with_tol(1e-8, warm_start=2), guess=guesses[i])
        assert warm[i].status == ref.status == O.SUCCESS, i
        assert abs(warm[i].iters - ref.iters) <= 1, (i, warm[i].iters, ref.iters)
        assert O.kkt_res(nxt[i], warm[i].sol) <= 1e-8 * 1.01, i
        assert rel(primal(warm[i].sol), primal(ref.sol)) <= 1e-6, i
