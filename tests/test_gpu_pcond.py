"""Partial condensing on the GPU (Section 3.5) against the oracle.

* the condensed QP the condensing kernel writes equals the oracle's condensed
  QP field by field (FP64, 1e-12 relative);
* with one stage per block the condensed path reproduces the plain batch
  solve bit for bit (condensing and expansion are then exact copies);
* full solves through condensing return, after the expansion kernel, a point
  of the original QP with KKT residual within the tolerance and the oracle's
  minimiser, in the iteration count of the oracle on the condensed QP.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from oracle import pcond as PC  # noqa: E402
from paper_2003_02547_amd import binding as B  # noqa: E402
from paper_2003_02547_amd import workloads as W  # noqa: E402

KEYS = ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u")
FIELDS = ("A", "B", "b", "Q", "S", "R", "q", "r", "lbu", "ubu", "lbx", "ubx", "D", "C", "lg", "ug")


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


def uneven_small(i):
    """Uneven-family instance with a short horizon (condensed stages fit the
    block kernel: inputs <= 64, general rows <= 64)."""
    rng = np.random.default_rng(np.random.SeedSequence([31, i]))
    nx = int(rng.integers(4, 13))
    nu = int(rng.integers(1, 9))
    return W.random_stable(rng, nx, nu, int(rng.integers(6, 15)))


def tiny(i):
    rng = np.random.default_rng(700 + i)
    return W.random_tiny(rng, int(rng.integers(3, 9)), nx_range=(1, 4), nu_range=(0, 3), ng_max=2)


def test_condensed_qp_matches_oracle():
    cases = [(W.mass_spring_chain8(0), 5), (W.mass_spring_chain8(1), 10), (W.mass_spring_chain8(2), 15),
             (W.mass_spring_chain4(1), 3)] + [(uneven_small(i), 3) for i in range(3)] + [(tiny(i), 2) for i in range(4)]
    say(f"condensed QP vs oracle: {len(cases)} instances, one batch per horizon")
    for N2 in sorted({c[1] for c in cases}):
        qps = [q for q, n2 in cases if n2 == N2]
        b = B.Batch(qps, B.default_arg(cond_N=N2)).load().solve().fetch_cond().sync()
        for i, qp in enumerate(qps):
            got = b.cond_qp(i)
            ref = PC.condense(qp, N2)
            assert got.N == ref.N and list(got.nx) == list(ref.nx) and list(got.nu) == list(ref.nu)
            for f in FIELDS:
                for n, (a, r) in enumerate(zip(getattr(got, f), getattr(ref, f))):
                    assert np.asarray(a).shape == np.asarray(r).shape, (N2, i, f, n)
                    assert rel(a, r) <= 1e-12, (N2, i, f, n, rel(a, r))
            for f in ("idxbu", "idxbx"):
                for n, (a, r) in enumerate(zip(getattr(got, f), getattr(ref, f))):
                    assert np.array_equal(a, r), (N2, i, f, n)


def test_one_stage_per_block_is_bitwise_the_plain_solve():
    qps = [W.mass_spring_chain4(s) for s in range(3)] + [tiny(i) for i in range(3)] + [W.mass_spring_chain8(0)]
    say("condensing with N2 = N vs plain batch: bitwise")
    plain = B.solve(qps)
    cond = B.solve(qps, B.default_arg(cond_N=1000))
    for i, (p, c) in enumerate(zip(plain, cond)):
        assert p.status == c.status and p.iters == c.iters, i
        for k in KEYS:
            assert np.array_equal(p.sol[k], c.sol[k]), (i, k)


@pytest.mark.parametrize("N2", [5, 10, 15])
def test_chain8_solves_through_condensing(N2):
    qps = [W.mass_spring_chain8(i) for i in range(8)]
    say(f"chain8 x8 through condensing to {N2} stages (FP64)")
    res = B.solve(qps, B.default_arg(cond_N=N2))
    for i, (q, r) in enumerate(zip(qps, res)):
        ref = O.solve(q, O.Arg.with_tol(1e-8))
        cref = O.solve(PC.condense(q, N2), O.Arg.with_tol(1e-8))
        if ref.status != O.SUCCESS:
            assert r.status != B.SUCCESS, i  # infeasible draw stays unsolved
            continue
        assert r.status == B.SUCCESS, (i, r.status, r.iters, r.res)
        assert abs(r.iters - cref.iters) <= 1, (i, r.iters, cref.iters)
        assert O.kkt_res(q, r.sol) <= 1e-8 + 1e-12, (i, O.kkt_res(q, r.sol))
        for k in ("u", "x"):
            assert rel(r.sol[k], ref.sol[k]) <= 1e-6, (i, k)


def test_mixed_size_batch_through_condensing():
    qps = [uneven_small(i) for i in range(4)] + [tiny(i) for i in range(4)] + [W.mass_spring_chain4(2)]
    N2 = 4  # some horizons are shorter: clipped per instance
    say("mixed-size batch through condensing, FP64 and mixed")
    res = B.solve(qps, B.default_arg(cond_N=N2))
    tol = 1e-6
    mixed = B.solve(qps, B.default_arg(B.MODE_MIXED, cond_N=N2, tol_stat=tol, tol_eq=tol, tol_ineq=tol, tol_comp=tol))
    for i, q in enumerate(qps):
        ref = O.solve(q, O.Arg.with_tol(1e-8))
        if ref.status != O.SUCCESS:
            continue
        r, m = res[i], mixed[i]
        assert r.status == B.SUCCESS, (i, r.status, r.res)
        assert O.kkt_res(q, r.sol) <= 1e-8 + 1e-12, i
        assert rel(r.sol["u"], ref.sol["u"]) <= 1e-6 and rel(r.sol["x"], ref.sol["x"]) <= 1e-6, i
        assert m.status == B.SUCCESS, (i, m.status, m.res, m.fell_back_f64)
        assert O.kkt_res(q, m.sol) <= tol * 1.01, (i, O.kkt_res(q, m.sol))


def test_condensing_batch_invariance_and_state_errors():
    qps = [W.mass_spring_chain8(i) for i in range(3)] + [uneven_small(5)]
    say("condensing: batch invariance, Newton entries refused")
    arg = B.default_arg(cond_N=6)
    full = B.solve(qps, arg)
    alone = B.solve([qps[2]], arg)[0]
    assert alone.iters == full[2].iters
    for k in KEYS:
        assert np.array_equal(alone.sol[k], full[2].sol[k]), k
    b = B.Batch(qps, arg).load()
    L = B.lib()
    assert L.oqp_batch_newton(b.h, 0.0) == B.ESTATE
    got = B.Qp(qps[0])  # any QP object: the state check comes first
    assert L.oqp_batch_get_cond_qp(b.h, 0, got.h) == B.ESTATE
    assert L.oqp_batch_fetch_cond(b.h) == B.ESTATE  # nothing solved yet
    b.sync()
