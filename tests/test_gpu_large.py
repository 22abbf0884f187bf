"""Parity of the block kernel's global-memory mode (stage blocks above 64)
with the FP64 oracle: the large-stage workload (nx = 128, nu = 32, N = 50,
32 general rows per stage) and smaller instances just above the LDS bound.

Bars as for the other kernels: Newton steps to 1e-8 relative (FP64) and
1e-6 after refinement (mixed); full solves to a host-evaluated KKT residual
<= 1e-8 and the oracle's primal solution to 1e-6 relative.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2003_02547_amd import binding as B  # noqa: E402
from paper_2003_02547_amd import workloads as W  # noqa: E402
from dense_ref import random_interior_iterate  # noqa: E402

KEYS = ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    B.lib()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b))))


def primal_err(sol, ref):
    return rel(np.concatenate([sol["u"], sol["x"]]), np.concatenate([ref["u"], ref["x"]]))


def medium(i, ng=4):
    """Stage block 72 (nx = 60, nu = 12) with general rows, short horizon."""
    rng = np.random.default_rng(np.random.SeedSequence([7, i]))
    return W.random_stable(rng, 60, 12, 8, ng=ng)


def newton_check(qps, tau, tol, arg=None, seed=3):
    rng = np.random.default_rng(seed)
    its = [random_interior_iterate(q, rng, scale=0.3) for q in qps]
    b = B.Batch(qps, arg).load()
    nv = B.lib().oqp_variant_count()
    for i, it in enumerate(its):
        assert b.variant(i)[0] >= nv + 4  # global-memory mode
        b.set_iterate(i, it)
    b.newton(tau).fetch().sync()
    for i, (q, it) in enumerate(zip(qps, its)):
        ref = O.newton_step(q, it, tau)
        got = b.step(i)
        for k in KEYS:
            assert rel(got[k], ref[k]) <= tol, (i, k, rel(got[k], ref[k]))


def test_global_mode_newton_step_fp64():
    qps = [medium(0), medium(1, ng=0), W.random_large_stage(0)]
    say("global mode newton: 2 medium + 1 large-stage")
    newton_check(qps, 0.02, 1e-8)


def test_global_mode_newton_step_mixed_refined():
    tol = 1e-6
    arg = B.default_arg(B.MODE_MIXED, tol_stat=tol, tol_eq=tol, tol_ineq=tol, tol_comp=tol)
    qps = [medium(2), W.random_large_stage(1)]
    say("global mode mixed newton")
    newton_check(qps, 0.05, 1e-6, arg=arg, seed=5)


def test_global_mode_solves_medium():
    qps = [medium(i) for i in range(4)]
    say("global mode solve: 4 medium")
    res = B.solve(qps)
    for i, (q, r) in enumerate(zip(qps, res)):
        ref = O.solve(q, O.Arg.with_tol(1e-8))
        assert ref.status == O.SUCCESS
        assert r.status == B.SUCCESS, (i, r.status, r.iters, r.res)
        assert O.kkt_res(q, r.sol) <= 1e-8 + 1e-12
        assert abs(ref.iters - r.iters) <= 1, (i, ref.iters, r.iters)
        assert primal_err(r.sol, ref.sol) <= 1e-6, (i, primal_err(r.sol, ref.sol))


def test_large_stage_solve_fp64_and_mixed():
    qp = W.random_large_stage(0)
    say("large-stage solve: FP64 and mixed vs oracle")
    ref = O.solve(qp, O.Arg.with_tol(1e-8))
    assert ref.status == O.SUCCESS
    r = B.solve([qp])[0]
    assert r.status == B.SUCCESS, (r.status, r.iters, r.res)
    assert O.kkt_res(qp, r.sol) <= 1e-8 + 1e-12
    assert abs(ref.iters - r.iters) <= 1
    assert primal_err(r.sol, ref.sol) <= 1e-6
    tol = 1e-8
    arg = B.default_arg(B.MODE_MIXED, tol_stat=tol, tol_eq=tol, tol_ineq=tol, tol_comp=tol)
    m = B.solve([qp], arg)[0]
    assert m.status == B.SUCCESS, (m.status, m.iters, m.res, m.fell_back_f64)
    assert O.kkt_res(qp, m.sol) <= 1e-8 + 1e-12
    assert primal_err(m.sol, ref.sol) <= 1e-6


def test_global_mode_batch_invariance_bitwise():
    qps = [medium(i) for i in range(3)] + [W.random_uneven(i) for i in range(5)] + [W.random_large_stage(2)]
    say("global mode invariance: mixed-size batch")
    full = B.solve(qps)
    for i in (1, 8):
        alone = B.solve([qps[i]])[0]
        assert alone.status == full[i].status and alone.iters == full[i].iters
        for k in KEYS:
            assert np.array_equal(full[i].sol[k], alone.sol[k]), (i, k)


def test_global_mode_workgroups_sharing_a_cu_bitwise():
    """More global-mode instances than CUs in one launch, and two such
    batches in flight on two streams: workgroups then share CUs (the build
    takes two waves per SIMD); every instance returns bitwise the result it
    has when solved alone."""
    distinct = [medium(i) for i in range(16)]
    qps = [distinct[i % 16] for i in range(320)]
    say("global mode: 2 x 320 instances in flight vs each instance alone")
    alone = [B.solve([q])[0] for q in distinct]
    copies = [B.Batch(qps, stream=torch.cuda.Stream()) for _ in range(2)]
    for c in copies:
        c.load()
    for c in copies:
        c.solve()
    torch.cuda.synchronize()
    for c in copies:
        res = c.fetch().sync().results()
        for i, r in enumerate(res):
            a = alone[i % 16]
            assert r.status == a.status and r.iters == a.iters, i
            for k in KEYS:
                assert np.array_equal(r.sol[k], a.sol[k], equal_nan=True), (i, k)
