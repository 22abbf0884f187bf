"""QR-based factorization on the GPU (mode robust of Section 4.2): the Riccati
factors come from Householder QR of [chol(Phi)'; U] instead of the Cholesky
factor of the normal matrix Phi + U'U.  The Newton step is the same in exact
arithmetic, so the reference is the oracle's Newton step and IPM.
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
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b))))


def tiny(i):
    rng = np.random.default_rng(1700 + i)
    return W.random_tiny(rng, int(rng.integers(2, 6)), nx_range=(1, 4), nu_range=(0, 3), ng_max=2)


def small_stable(i):
    rng = np.random.default_rng(np.random.SeedSequence([41, i]))
    return W.random_stable(rng, int(rng.integers(4, 17)), int(rng.integers(1, 9)), int(rng.integers(5, 30)))


def test_robust_newton_step():
    qps = [tiny(i) for i in range(6)] + [W.mass_spring_chain4(1), W.mass_spring_chain8(3), small_stable(0)]
    rng = np.random.default_rng(77)
    its = [random_interior_iterate(q, rng, scale=0.5) for q in qps]
    say("robust-mode Newton step vs oracle")
    b = B.Batch(qps, B.default_arg(B.MODE_ROBUST)).load()
    nv = B.lib().oqp_variant_count()
    for i, it in enumerate(its):
        assert b.variant(i)[0] < nv
        b.set_iterate(i, it)
    b.newton(0.02).fetch().sync()
    for i, (q, it) in enumerate(zip(qps, its)):
        ref = O.newton_step(q, it, 0.02)
        got = b.step(i)
        for k in KEYS:
            assert rel(got[k], ref[k]) <= 1e-8, (i, k, rel(got[k], ref[k]))


def test_robust_solves_follow_the_oracle():
    qps = [W.mass_spring_chain4(s) for s in range(4)] + [W.mass_spring_chain8(i) for i in range(6)] + \
        [small_stable(i) for i in range(4)] + [tiny(i) for i in range(4)]
    say("robust-mode solves vs oracle")
    res = B.solve(qps, B.default_arg(B.MODE_ROBUST))
    plain = B.solve(qps)
    for i, (q, r) in enumerate(zip(qps, res)):
        ref = O.solve(q, O.Arg.with_tol(1e-8))
        assert r.status == ref.status, (i, r.status, ref.status)
        if ref.status != O.SUCCESS:
            continue
        assert abs(r.iters - ref.iters) <= 1, (i, r.iters, ref.iters)
        assert O.kkt_res(q, r.sol) <= 1e-8 + 1e-12
        for k in ("u", "x"):
            assert rel(r.sol[k], ref.sol[k]) <= 1e-6, (i, k)
        # same Newton steps as the Cholesky path up to rounding
        assert abs(r.iters - plain[i].iters) <= 1, (i, r.iters, plain[i].iters)
