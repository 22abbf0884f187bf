"""The wide-stage kernel (stages beyond the block kernel's limits: more than
64 inputs, more than 64 general rows, or more than 256 constraint slots)
and full condensing through it (Section 3.5 with one block; the dense
Cholesky factorization of the condensed Hessian, Section 3.3), against the
oracles:

* Newton steps at random interior iterates equal the OCP oracle's;
* solves reach the oracle's minimiser with the oracle's status and
  iteration count (within one), KKT residual on the host within tolerance;
* a batch solved through full condensing (cond_N = 1) returns the original
  QP's minimiser: the OCP oracle on the uncondensed QP and the dense oracle
  (full condensing, dense Cholesky IPM) agree with it, and the condensed QP
  the GPU builds equals the oracle's;
* wide instances share a batch with one-wave and block-kernel instances
  without changing anyone's result.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import dense as D  # noqa: E402
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


def primal_err(sol, ref):
    return rel(np.concatenate([sol["u"], sol["x"]]), np.concatenate([ref["u"], ref["x"]]))


def n_rows(qp):
    return sum(len(i) for i in qp.idxbu) + sum(len(i) for i in qp.idxbx) + sum(np.asarray(d).shape[0] for d in qp.D)


def interior(qp, rng, scale=0.4):
    nc = n_rows(qp)
    return dict(u=rng.standard_normal(sum(qp.nu)) * scale, x=rng.standard_normal(sum(qp.nx)) * scale,
                pi=rng.standard_normal(sum(qp.nx[1:])) * scale, lam_l=rng.uniform(0.1, 2.0, nc),
                lam_u=rng.uniform(0.1, 2.0, nc), t_l=rng.uniform(0.1, 2.0, nc), t_u=rng.uniform(0.1, 2.0, nc))


def as_ocp(ns):
    """The oracle's condensed QP (a namespace of the same fields) as an OCP QP
    object the batch accepts."""
    f = ("A", "B", "b", "Q", "S", "R", "q", "r", "idxbu", "lbu", "ubu", "idxbx", "lbx", "ubx", "D", "C", "lg", "ug")
    return W.OcpQp(ns.N, list(ns.nx), list(ns.nu), *[list(getattr(ns, k)) for k in f])


def wide_cases():
    """One instance per way of exceeding the block kernel: the fully
    condensed 8-mass chain (210 inputs, 232 general rows), more than 64
    inputs, more than 64 general rows, and inputs at the terminal stage."""
    rng = lambda s: np.random.default_rng(np.random.SeedSequence([61, s]))
    return [as_ocp(PC.condense(W.mass_spring_chain8(4), 1)),
            W.random_stable(rng(1), 12, 70, 4),
            W.random_stable(rng(2), 10, 6, 5, ng=80),
            W.random_tiny(rng(3), 3, nx_range=(2, 4), nu_range=(66, 70), ng_max=2)]


def test_wide_instances_take_the_wide_kernel():
    qps = wide_cases()
    b = B.Batch(qps)
    nv = B.lib().oqp_variant_count()
    for i in range(len(qps)):
        assert b.variant(i)[0] == nv + 6, (i, b.variant(i))


def test_wide_newton_step_matches_oracle():
    qps = wide_cases()
    rng = np.random.default_rng(5)
    its = [interior(q, rng) for q in qps]
    say("wide kernel: Newton steps vs oracle")
    b = B.Batch(qps).load()
    for i, it in enumerate(its):
        b.set_iterate(i, it)
    for tau in (0.0, 0.05):
        b.newton(tau).fetch().sync()
        for i, (q, it) in enumerate(zip(qps, its)):
            ref = O.newton_step(q, it, tau)
            got = b.step(i)
            for k in KEYS:
                assert rel(got[k], ref[k]) <= 1e-8, (i, tau, k, rel(got[k], ref[k]))


def test_wide_solves_follow_the_oracle():
    qps = wide_cases()
    say("wide kernel: solves vs oracle")
    res = B.solve(qps)
    for i, (q, r) in enumerate(zip(qps, res)):
        ref = O.solve(q, O.Arg.with_tol(1e-8))
        assert r.status == ref.status, (i, r.status, ref.status, r.iters, r.res)
        if ref.status != O.SUCCESS:
            continue
        assert abs(r.iters - ref.iters) <= 1, (i, r.iters, ref.iters)
        assert O.kkt_res(q, r.sol) <= 1e-8 + 1e-12, (i, O.kkt_res(q, r.sol))
        assert primal_err(r.sol, ref.sol) <= 1e-6, (i, primal_err(r.sol, ref.sol))


def test_full_condensing_of_the_chain():
    """The 8-mass chain (nx = 16, nu = 7, N = 30) fully condensed on the GPU
    and solved by the wide kernel: the original QP's minimiser."""
    qps = [W.mass_spring_chain8(i) for i in range(6)]
    say("8-mass chain x6, full condensing (cond_N = 1) vs the OCP and dense oracles")
    b = B.Batch(qps, B.default_arg(cond_N=1)).load().solve().fetch_cond().fetch().sync()
    res = b.results()
    for i, (q, r) in enumerate(zip(qps, res)):
        cq = PC.condense(q, 1)
        got = b.cond_qp(i)
        for f in FIELDS:
            for n, (a, c) in enumerate(zip(getattr(got, f), getattr(cq, f))):
                assert rel(a, c) <= 1e-12, (i, f, n, rel(a, c))
        ref = O.solve(q, O.Arg.with_tol(1e-8))
        cref = O.solve(cq, O.Arg.with_tol(1e-8))
        if ref.status != O.SUCCESS:
            assert r.status != B.SUCCESS, i
            continue
        assert r.status == B.SUCCESS, (i, r.status, r.iters, r.res)
        assert abs(r.iters - cref.iters) <= 1, (i, r.iters, cref.iters)
        assert O.kkt_res(q, r.sol) <= 1e-8 + 1e-12, (i, O.kkt_res(q, r.sol))
        assert primal_err(r.sol, ref.sol) <= 1e-6, (i, primal_err(r.sol, ref.sol))
        dst, _, dsol, _ = D.solve(q, tol=1e-8)
        assert dst == 0
        assert primal_err(r.sol, dsol) <= 1e-6, (i, primal_err(r.sol, dsol))


def test_wide_instances_share_a_batch():
    wide = wide_cases()
    small = [W.mass_spring_chain4(1), W.mass_spring_chain8(2),
             W.random_stable(np.random.default_rng(7), 40, 12, 6)]
    say("wide kernel next to one-wave and block-kernel groups: bitwise as alone")
    mixed = B.solve(small[:1] + wide[:2] + small[1:] + wide[2:])
    alone_w = B.solve(wide)
    alone_s = B.solve(small)
    order = [("s", 0), ("w", 0), ("w", 1), ("s", 1), ("s", 2), ("w", 2), ("w", 3)]
    for m, (kind, j) in zip(mixed, order):
        a = (alone_s if kind == "s" else alone_w)[j]
        assert m.status == a.status and m.iters == a.iters, (kind, j)
        for k in KEYS:
            assert np.array_equal(m.sol[k], a.sol[k]), (kind, j, k)
