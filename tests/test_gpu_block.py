"""Parity of the 256-thread block kernel with the FP64 oracle.

The one-wave bound is set to 0 for this module so that every instance,
small ones included, runs on the block kernel.  Bars as for the one-wave
kernel: Newton steps to 1e-9 relative (FP64) and 1e-6 after refinement
(mixed); FP64 solves to a host-evaluated KKT residual <= 1e-8 and the
oracle's primal solution to 1e-6 relative, iteration counts within one.
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
def _block_only():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    old = B.set_wave_max(0)
    yield
    B.set_wave_max(old)


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b))))


def primal_err(sol, ref):
    return rel(np.concatenate([sol["u"], sol["x"]]), np.concatenate([ref["u"], ref["x"]]))


def newton_check(qps, its, tau, tol, arg=None):
    b = B.Batch(qps, arg).load()
    nv = B.lib().oqp_variant_count()
    for i, it in enumerate(its):
        assert b.variant(i)[0] >= nv  # block kernel
        b.set_iterate(i, it)
    b.newton(tau).fetch().sync()
    for i, (q, it) in enumerate(zip(qps, its)):
        ref = O.newton_step(q, it, tau)
        got = b.step(i)
        for k in KEYS:
            assert rel(got[k], ref[k]) <= tol, (i, k, rel(got[k], ref[k]), b.variant(i))


def test_block_newton_step_tiny_general_rows():
    qps = []
    for s in range(24):
        rng = np.random.default_rng(900 + s)
        qps.append(W.random_tiny(rng, int(rng.integers(1, 6)), ng_max=3,
                                 x0_mode=["box", "free", "eliminated"][s % 3]))
    rng = np.random.default_rng(3)
    its = [random_interior_iterate(q, rng) for q in qps]
    say("block newton: 24 tiny")
    newton_check(qps, its, 0.07, 1e-9)


def test_block_newton_step_chain8_and_large():
    qps = [W.mass_spring_chain8(3)]
    qps += [q for q in (W.random_uneven(i) for i in range(120)) if q.nx[1] + q.nu[0] > 40][:4]
    rng = np.random.default_rng(11)
    its = [random_interior_iterate(q, rng, scale=0.4) for q in qps]
    say("block newton: chain8 + 4 large uneven")
    newton_check(qps, its, 0.02, 1e-8)


def check_solves(qps, res, tol=1e-8):
    for i, (q, r) in enumerate(zip(qps, res)):
        ref = O.solve(q, O.Arg.with_tol(tol))
        if ref.status != O.SUCCESS:
            assert r.status != B.SUCCESS, i
            continue
        assert r.status == B.SUCCESS, (i, r.status, r.iters, r.res)
        assert O.kkt_res(q, r.sol) <= tol + 1e-12, i
        assert abs(ref.iters - r.iters) <= 1, (i, ref.iters, r.iters)
        assert primal_err(r.sol, ref.sol) <= 1e-6, (i, primal_err(r.sol, ref.sol))


def test_block_solves_chain4_and_tiny():
    qps = [W.mass_spring_chain4(s) for s in range(1, 11)]
    rng = np.random.default_rng(77)
    qps += [W.random_tiny(rng, int(rng.integers(1, 6)), ng_max=2) for _ in range(10)]
    say("block solve: chain4 x10 + tiny x10")
    check_solves(qps, B.solve(qps))


def test_block_solves_chain8_sampled():
    qps = [W.mass_spring_chain8(i) for i in range(64)]
    say("block solve: chain8 x64, 12 sampled")
    res = B.solve(qps)
    idx = list(range(0, 64, 6))
    check_solves([qps[i] for i in idx], [res[i] for i in idx])
    assert sum(r.status == B.SUCCESS for r in res) >= 60


def test_block_matches_wave_kernel():
    """Same instances through both kernel families: same iteration counts
    (within one) and primal solutions within 1e-6 relative."""
    qps = [W.mass_spring_chain8(i) for i in range(16)]
    say("block vs wave: chain8 x16")
    blk = B.solve(qps)
    old = B.set_wave_max(24)
    try:
        wav = B.solve(qps)
    finally:
        B.set_wave_max(old)
    for i, (a, b) in enumerate(zip(blk, wav)):
        assert a.status == b.status, i
        if a.status == B.SUCCESS:
            assert abs(a.iters - b.iters) <= 1, (i, a.iters, b.iters)
            assert primal_err(a.sol, b.sol) <= 1e-6, i


def test_block_uneven_sizes_one_launch_bitwise_invariant():
    """Instances of different sizes share one block launch; each result is
    bitwise the one it gets alone."""
    qps = [W.random_uneven(i) for i in range(16)]
    say("block invariance: uneven x16")
    full = B.solve(qps)
    for i in (0, 5, 11):
        alone = B.solve([qps[i]])[0]
        assert alone.status == full[i].status and alone.iters == full[i].iters
        for k in KEYS:
            assert np.array_equal(full[i].sol[k], alone.sol[k]), (i, k)
    ok = 0
    for i in range(0, 16, 3):
        ref = O.solve(qps[i], O.Arg.with_tol(1e-8))
        if ref.status == O.SUCCESS:
            assert full[i].status == B.SUCCESS
            assert primal_err(full[i].sol, ref.sol) <= 1e-6
            ok += 1
    assert ok >= 4


def mixed_arg(tol=1e-6, **kw):
    return B.default_arg(B.MODE_MIXED, tol_stat=tol, tol_eq=tol, tol_ineq=tol, tol_comp=tol, **kw)


def test_block_mixed_refined_newton_step():
    qps = [W.mass_spring_chain8(5)]
    for s in range(8):
        rng = np.random.default_rng(1700 + s)
        qps.append(W.random_tiny(rng, int(rng.integers(1, 5)), ng_max=2))
    rng = np.random.default_rng(9)
    its = [random_interior_iterate(q, rng, scale=0.5) for q in qps]
    say("block mixed newton")
    newton_check(qps, its, 0.05, 1e-6, arg=mixed_arg())


def test_block_mixed_solves():
    qps = [W.mass_spring_chain8(i) for i in range(24)] + [W.random_uneven(i) for i in range(8)]
    say("block mixed solve: chain8 x24 + uneven x8 at tol 1e-8")
    res = B.solve(qps, mixed_arg(1e-8))
    for i in range(0, len(qps), 4):
        ref = O.solve(qps[i], O.Arg.with_tol(1e-8))
        if ref.status != O.SUCCESS:
            continue
        r = res[i]
        assert r.status == B.SUCCESS, (i, r.status, r.res, r.fell_back_f64)
        assert O.kkt_res(qps[i], r.sol) <= 1e-8 + 1e-12
        assert primal_err(r.sol, ref.sol) <= 1e-6, i
