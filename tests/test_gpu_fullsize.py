"""Parity at the workloads' full sizes, in the launch configurations the
benchmark times, checked instance by instance against the oracle (every
instance where the oracle finishes the batch in seconds, samples of the
large-stage batch):

* the 8-mass batch of 1024, mixed path (refined to KKT 1e-6);
* the uneven batch of 4096 (nx 4..48, nu 1..16, N 10..100) with its kernel
  groups on three extra streams, FP64 and mixed;
* the large-stage batch of 256 (nx 128, nu 32, N 50, 32 general rows): FP64
  with refinement of the prediction-centering-correction direction to 1e-8
  (every instance), without it on the instances where the plain iteration
  stalls (the oracle stalls there too), mixed to the metric's tolerance.

Host-side bars: KKT residual of every returned point, evaluated by the
oracle's residual routine (FP64 path 1e-8, mixed 1e-6), statuses, and the
primal solution against the oracle's: 1e-6 where both run the same arguments
in FP64, and for the mixed path when it is run to 1e-8; a point at KKT 1e-6
can sit ~1e-3 from the minimiser on these chains, so the mixed path at the
metric's tolerance is held to the KKT bar (its largest primal error stated,
with a sanity bound).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2003_02547_amd import binding as B  # noqa: E402
from paper_2003_02547_amd import workloads as W  # noqa: E402
from oracle_pool import kkt_many, solve_many  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    B.lib()


def primal_err(sol, ref):
    a = np.concatenate([sol["u"], sol["x"]])
    b = np.concatenate([ref["u"], ref["x"]])
    return float(np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b))))


def tol_arg(mode, tol):
    return B.default_arg(mode, tol_stat=tol, tol_eq=tol, tol_ineq=tol, tol_comp=tol)


@pytest.mark.parametrize("tol", [1e-6, 1e-8])
def test_chain8_full_batch_mixed_every_instance(tol):
    """Mixed path on all 1024: the two infeasible instances fail, every other
    point meets the KKT bar on the host; the primal error against the
    oracle's FP64 solution at 1e-8 is stated.  A KKT residual bounds that
    error only through the conditioning: at the metric's 1e-6 a point can sit
    ~1e-3 from the minimiser on these chains, at 1e-8 ~1.5e-5 (the FP64 path
    too); held to 2e-3 and 1e-4 as sanity bounds."""
    qps = [W.mass_spring_chain8(i) for i in range(1024)]
    say(f"8-mass x1024, mixed path to {tol}, every instance vs oracle")
    res = B.solve(qps, tol_arg(B.MODE_MIXED, tol))
    assert [i for i, r in enumerate(res) if r.status != B.SUCCESS] == [222, 350]
    good = [i for i in range(1024) if i not in (222, 350)]
    kkt = kkt_many(qps, [r.sol for r in res], good)
    worst = max(kkt, key=kkt.get)
    assert kkt[worst] <= tol * 1.01, (worst, kkt[worst])
    refs = solve_many(qps, good, O.Arg.with_tol(1e-8))
    err = {i: primal_err(res[i].sol, refs[i].sol) for i in good}
    worst = max(err, key=err.get)
    say(f"mixed to {tol}: max primal rel err vs oracle {err[worst]:.2e} (instance {worst})")
    assert err[worst] <= (2e-3 if tol > 1e-8 else 1e-4), (worst, err[worst])


@pytest.mark.parametrize("mode", [B.MODE_F64, B.MODE_MIXED])
def test_uneven_4096_on_extra_streams_every_instance(mode):
    """Every instance of the uneven batch: host KKT residual of the returned
    point (FP64 1e-8, mixed 1e-6) and the primal solution against the
    oracle's FP64 solution (same arguments): FP64 to 1e-6 with an iteration
    count within one of the oracle's; mixed at the metric's tolerance held to
    the KKT bar, its largest primal error stated."""
    qps = [W.random_uneven(i) for i in range(4096)]
    say(f"uneven x4096 on 3 extra streams, mode {mode}, every instance vs oracle")
    arg = B.default_arg() if mode == B.MODE_F64 else tol_arg(B.MODE_MIXED, 1e-6)
    b = B.Batch(qps, arg, streams=3).load().solve().fetch().sync()
    res = b.results()
    assert [i for i, r in enumerate(res) if r.status != B.SUCCESS] == []
    groups = {b.variant(i)[0] for i in range(4096)}
    assert len(groups) >= 8
    bar = 1e-8 if mode == B.MODE_F64 else 1e-6
    kkt = kkt_many(qps, [r.sol for r in res], range(4096))
    worst = max(kkt, key=kkt.get)
    assert kkt[worst] <= bar * 1.01, (worst, kkt[worst])
    refs = solve_many(qps, range(4096), O.Arg.with_tol(1e-8))
    assert all(refs[i].status == O.SUCCESS for i in range(4096))
    err = {i: primal_err(res[i].sol, refs[i].sol) for i in range(4096)}
    worst = max(err, key=err.get)
    say(f"uneven x4096 mode {mode}: max primal rel err vs oracle {err[worst]:.2e} (instance {worst})")
    if mode == B.MODE_F64:
        it_diff = {i: abs(refs[i].iters - res[i].iters) for i in range(4096)}
        assert max(it_diff.values()) <= 1, max(it_diff.items(), key=lambda kv: kv[1])
        assert err[worst] <= 1e-6, (worst, err[worst])
    else:
        assert err[worst] <= 2e-3, (worst, err[worst])


# Instances of the large-stage batch on which the plain FP64 iteration stalls
# before KKT 1e-8 in the oracle (stationarity residual rising again in late
# iterations); with refinement of the prediction-centering-correction
# direction every instance converges.
LARGE_STALL = (1, 115)


def test_large_stage_256_fp64_refined_to_1e8():
    """Every instance of the batch to KKT 1e-8 on the FP64 path with up to 4
    refinement corrections per direction (the configuration the benchmark
    times); the KKT residual of every returned point evaluated on the host,
    statuses and primal solutions compared with the oracle (same arguments)
    on a sample that holds the instances where refinement is needed."""
    qps = [W.random_large_stage(i) for i in range(256)]
    say("large-stage x256, FP64 with refinement (ir_max 4) to 1e-8")
    arg = tol_arg(B.MODE_F64, 1e-8)
    arg.ir_max = 4
    res = B.solve(qps, arg)
    bad = [i for i, r in enumerate(res) if r.status != B.SUCCESS]
    assert bad == [], bad
    kkt = kkt_many(qps, [r.sol for r in res], range(256))
    worst = max(kkt, key=kkt.get)
    assert kkt[worst] <= 1e-8 * 1.01, (worst, kkt[worst])
    assert sum(r.ir_steps for r in res) > 0
    picks = list(LARGE_STALL) + [0, 64, 131, 200]
    refs = solve_many(qps, picks, O.Arg.with_tol(1e-8, ir_max=4))
    for i in picks:
        assert refs[i].status == O.SUCCESS, i
        assert abs(refs[i].iters - res[i].iters) <= 2, (i, refs[i].iters, res[i].iters)
        assert primal_err(res[i].sol, refs[i].sol) <= 1e-6, (i, primal_err(res[i].sol, refs[i].sol))


def test_large_stage_stall_without_refinement_matches_oracle():
    """Without refinement both sides stop short of 1e-8 on the instances
    named above (the breakdown is the method's, not the kernel's)."""
    qps = [W.random_large_stage(i) for i in LARGE_STALL]
    say("large-stage stall instances, FP64 without refinement to 1e-8")
    res = B.solve(qps, tol_arg(B.MODE_F64, 1e-8))
    refs = solve_many(qps, list(range(len(qps))), O.Arg.with_tol(1e-8))
    for k, i in enumerate(LARGE_STALL):
        assert refs[k].status != O.SUCCESS, i
        assert res[k].status != B.SUCCESS, (i, res[k].status, res[k].res)


def test_large_stage_256_mixed_sampled():
    """Mixed path at the metric's tolerance: every returned point held to KKT
    1e-6 on the host; the primal error against the oracle's FP64 solution
    (run to 1e-8 with refinement) stated per sampled result."""
    qps = [W.random_large_stage(i) for i in range(256)]
    say("large-stage x256, mixed at 1e-6")
    res = B.solve(qps, tol_arg(B.MODE_MIXED, 1e-6))
    bad = [i for i, r in enumerate(res) if r.status != B.SUCCESS]
    assert bad == [], bad
    kkt = kkt_many(qps, [r.sol for r in res], range(256))
    worst = max(kkt, key=kkt.get)
    assert kkt[worst] <= 1e-6 * 1.01, (worst, kkt[worst])
    picks = list(LARGE_STALL) + [0, 131]
    refs = solve_many(qps, picks, O.Arg.with_tol(1e-8, ir_max=4))
    errs = {i: primal_err(res[i].sol, refs[i].sol) for i in picks}
    say(f"mixed primal rel err vs oracle: {errs}")
    assert max(errs.values()) <= 1e-4, errs
