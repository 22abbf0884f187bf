"""The array algorithm (Section 4.2, modes robust and balance) on the block
kernel: stage blocks up to 32 and up to 64 with the stage matrices in LDS,
and the global-memory mode above 64.  The Newton step of the QR-based
factorization equals the Cholesky one in exact arithmetic, so the reference
is the oracle's Newton step and IPM, as for the one-wave builds.
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


@pytest.fixture
def block_only():
    """Every instance on the block kernel."""
    old = B.set_wave_max(0)
    yield
    B.set_wave_max(old)


def rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b))))


def primal_err(sol, ref):
    return rel(np.concatenate([sol["u"], sol["x"]]), np.concatenate([ref["u"], ref["x"]]))


def stable(i, nx, nu, N, ng=0):
    rng = np.random.default_rng(np.random.SeedSequence([43, i]))
    return W.random_stable(rng, nx, nu, N, ng=ng)


def shapes():
    """One instance per block build: up to 32 (with and without general
    rows), up to 64, and the global-memory mode (stage block 72)."""
    return [stable(0, 12, 4, 12), stable(1, 20, 8, 10, ng=3), stable(2, 40, 12, 8), stable(3, 36, 10, 8, ng=5),
            stable(4, 60, 12, 6, ng=4), W.mass_spring_chain8(5)]


@pytest.mark.parametrize("mode", [B.MODE_ROBUST, B.MODE_BALANCE])
def test_block_newton_step_array_algorithm(block_only, mode):
    qps = shapes()
    rng = np.random.default_rng(91)
    its = [random_interior_iterate(q, rng, scale=0.4) for q in qps]
    say(f"block kernel, mode {mode}: Newton step vs oracle")
    # robust: the array algorithm alone (no refinement); balance: forced to it
    # by a check that always fails (ir_tol = 0)
    arg = B.default_arg(mode, ir_max=0, ir_tol=0.0)
    b = B.Batch(qps, arg).load()
    nv = B.lib().oqp_variant_count()
    for i, it in enumerate(its):
        assert b.variant(i)[0] >= nv
        b.set_iterate(i, it)
    b.newton(0.03).fetch().sync()
    for i, (q, it) in enumerate(zip(qps, its)):
        ref = O.newton_step(q, it, 0.03)
        got = b.step(i)
        for k in KEYS:
            assert rel(got[k], ref[k]) <= 1e-8, (i, k, rel(got[k], ref[k]))


def test_block_robust_solves_follow_the_oracle(block_only):
    qps = shapes() + [W.mass_spring_chain4(2)]
    say("block kernel, mode robust: solves vs oracle")
    res = B.solve(qps, B.default_arg(B.MODE_ROBUST))
    for i, (q, r) in enumerate(zip(qps, res)):
        ref = O.solve(q, O.Arg.with_tol(1e-8, ir_max=4))
        assert ref.status == O.SUCCESS
        assert r.status == B.SUCCESS, (i, r.status, r.iters, r.res)
        assert O.kkt_res(q, r.sol) <= 1e-8 + 1e-12
        assert abs(r.iters - ref.iters) <= 1, (i, r.iters, ref.iters)
        assert primal_err(r.sol, ref.sol) <= 1e-6, (i, primal_err(r.sol, ref.sol))


def test_block_balance_check_limits(block_only):
    """Balance mode through the two limits of its check: a check that always
    passes (ir_tol huge, no refinement) is the Cholesky path (to rounding of a
    different build); a check
    that always fails factors every iteration with the array algorithm, and
    the solve still reaches the oracle's minimiser."""
    qps = shapes()
    say("block kernel, mode balance: limits of the check")
    plain = B.solve(qps)
    never = B.solve(qps, B.default_arg(B.MODE_BALANCE, ir_tol=1e300, ir_max=0))
    for i, (p, n) in enumerate(zip(plain, never)):
        assert n.qr_refactors == 0 and n.ir_steps == 0, i
        assert n.status == p.status and n.iters == p.iters, (i, n.status, p.status, n.iters, p.iters)
        for k in KEYS:
            assert rel(n.sol[k], p.sol[k]) <= 1e-12, (i, k, rel(n.sol[k], p.sol[k]))
    always = B.solve(qps, B.default_arg(B.MODE_BALANCE, ir_tol=0.0))
    for i, (q, r) in enumerate(zip(qps, always)):
        ref = O.solve(q, O.Arg.with_tol(1e-8, ir_max=2))
        assert ref.status == O.SUCCESS
        assert r.status == B.SUCCESS, (i, r.status, r.res)
        assert r.qr_refactors == r.iters, (i, r.qr_refactors, r.iters)
        assert O.kkt_res(q, r.sol) <= 1e-8 + 1e-12
        assert primal_err(r.sol, ref.sol) <= 1e-6, (i, primal_err(r.sol, ref.sol))


def test_large_stage_array_algorithm_solves():
    """The large-stage workload (global-memory mode) in both modes to KKT
    1e-8: instance 1 is one where the plain Cholesky iteration stalls."""
    qps = [W.random_large_stage(i) for i in (0, 1)]
    say("large-stage instances 0 and 1, modes robust and balance, to 1e-8")
    for mode in (B.MODE_ROBUST, B.MODE_BALANCE):
        res = B.solve(qps, B.default_arg(mode))
        for i, (q, r) in enumerate(zip(qps, res)):
            assert r.status == B.SUCCESS, (mode, i, r.status, r.iters, r.res)
            assert O.kkt_res(q, r.sol) <= 1e-8 * 1.01, (mode, i)
