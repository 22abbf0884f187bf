"""Absolute formulation on the GPU (Section 3.2, eq:alg:pdipm:abs; mode
speed_abs of Section 4.2) against the oracle.

* the Newton step through the absolute system equals the oracle's (and the
  delta step) on the one-wave and block kernels;
* the first iterations follow the delta formulation's iterates;
* full solves exit on the duality measure in the oracle's iteration count,
  near its point (the absolute formulation is limited by cancellation near
  the solution, so the bar is looser than the delta path's), and the
  reported residual norms are those of the returned point.
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
    rng = np.random.default_rng(1300 + i)
    return W.random_tiny(rng, int(rng.integers(2, 6)), nx_range=(1, 4), nu_range=(0, 3), ng_max=2)


@pytest.mark.parametrize("kernel", ["wave", "block"])
def test_abs_newton_step(kernel):
    qps = [tiny(i) for i in range(6)] + [W.mass_spring_chain4(1)]
    rng = np.random.default_rng(31)
    its = [random_interior_iterate(q, rng, scale=0.5) for q in qps]
    say(f"absolute-formulation Newton step, {kernel} kernel")
    old = B.set_wave_max(64 if kernel == "wave" else 0)
    try:
        b = B.Batch(qps, B.default_arg(B.MODE_ABS)).load()
        for i, it in enumerate(its):
            b.set_iterate(i, it)
        b.newton(0.05).fetch().sync()
        for i, (q, it) in enumerate(zip(qps, its)):
            ref = O.newton_step(q, it, 0.05, abs_form=True)
            got = b.step(i)
            for k in KEYS:
                assert rel(got[k], ref[k]) <= 1e-8, (i, k, rel(got[k], ref[k]))
    finally:
        B.set_wave_max(old)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_first_iterations_follow_the_delta_formulation(k):
    qps = [W.mass_spring_chain8(i) for i in range(4)] + [W.random_uneven(i) for i in range(3)]
    say(f"absolute vs delta, {k} iterations")
    a = B.solve(qps, B.default_arg(B.MODE_ABS, iter_max=k))
    d = B.solve(qps, B.default_arg(iter_max=k))
    for i, (x, y) in enumerate(zip(a, d)):
        assert x.iters == y.iters == k, i
        for key in KEYS:
            assert rel(x.sol[key], y.sol[key]) <= 1e-9, (k, i, key)


def test_abs_solves_follow_the_oracle():
    qps = [W.mass_spring_chain4(s) for s in range(3)] + [W.mass_spring_chain8(i) for i in range(4)] + \
        [W.random_uneven(i) for i in range(3)]
    tol = 1e-6
    say("absolute-formulation solves vs oracle")
    res = B.solve(qps, B.default_arg(B.MODE_ABS, tol_comp=tol))
    for i, (q, r) in enumerate(zip(qps, res)):
        ref = O.solve(q, O.Arg.with_tol(tol, abs_form=1))
        assert r.status == ref.status, (i, r.status, ref.status)
        if ref.status != O.SUCCESS:
            continue
        assert r.mu <= tol and abs(r.iters - ref.iters) <= 1, (i, r.mu, r.iters, ref.iters)
        for k in ("u", "x"):
            assert rel(r.sol[k], ref.sol[k]) <= 1e-4, (i, k, rel(r.sol[k], ref.sol[k]))
        # stat.res: the residual norms at the returned point
        _, norms, _ = O.residuals(q, r.sol)
        assert np.allclose(r.res, norms, rtol=1e-6, atol=1e-13), (i, r.res, norms)
