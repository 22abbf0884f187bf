"""Pins of the oracle's iterative refinement (Section 3.4) and of its use on
the prediction-centering-correction direction (Section 4.2).

* A refined Newton step, factored with a primal regularization, reaches the
  step of the unregularized system (dense LU of eq:alg:pdipm:delta): the
  refinement residual is formed with the matrix K itself, so the corrections
  offset the regularization (Section 4.2 says this of the regularization).
  Without refinement the regularized step stays off by O(reg).
* On an iterate whose barrier weights span many orders of magnitude (late
  IPM iterations, Section 3.4), the refined step satisfies the full Newton
  system better than the unrefined one (at least by half here), measured by
  a dense evaluation of K d + r.
* On the large-stage workload (nx 128, nu 32, N 50, 32 general rows) the
  plain FP64 iteration stalls before the 1e-8 tolerance, and with refinement
  of that direction it reaches it; the returned point's KKT residual is
  evaluated independently in dense form.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_02547_amd import workloads as W
from dense_ref import DenseQp, random_interior_iterate

FLAT = ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u")


def _rel(a, b):
    err = 0.0
    for k in FLAT:
        x, y = np.asarray(a[k]), np.asarray(b[k])
        if x.size:
            err = max(err, float(np.max(np.abs(x - y)) / max(1.0, np.max(np.abs(y)))))
    return err


def _tiny(seed, **kw):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 5))
    return W.random_tiny(rng, N, **kw), rng


def _dense_ir_norm(dq, it, tau, step):
    """||K d + r||_inf of the full 4-block system, in dense form."""
    rg, rb, rd, rm = dq.residual(it, tau)
    K = dq.kkt_matrix(it)
    y, pi, lam, t = dq.stack(step)
    d = np.concatenate([y, pi, lam, t])
    return float(np.max(np.abs(K @ d + np.concatenate([rg, rb, rd, rm]))))


@pytest.mark.parametrize("seed", range(8))
def test_refinement_offsets_regularization(seed):
    qp, rng = _tiny(seed, ng_max=2)
    dq = DenseQp(qp)
    it = random_interior_iterate(qp, rng)
    tau = float(rng.uniform(0.0, 0.3))
    ref = dq.newton_step(it, tau)
    reg = 1e-3
    plain = O.newton_step(qp, it, tau, reg=reg)
    refined, kept = O.newton_step_refined(qp, it, tau, reg=reg, ir_max=30, ir_tol=1e-14)
    assert _rel(plain, ref) > 1e-7, "the regularized step must differ from the exact one"
    assert kept >= 1
    assert _rel(refined, ref) <= 1e-9, (_rel(refined, ref), kept)
    # no regularization, no refinement: the plain step
    same, kept0 = O.newton_step_refined(qp, it, tau, reg=0.0, ir_max=0)
    assert kept0 == 0
    assert _rel(same, O.newton_step(qp, it, tau)) == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_refined_step_residual_lower_on_extreme_weights(seed):
    qp, rng = _tiny(seed, ng_max=2)
    dq = DenseQp(qp)
    it = random_interior_iterate(qp, rng)
    # late-iteration weights: half the one-sided rows nearly active (t tiny,
    # lam ~ 1), the other half nearly inactive (lam tiny, t ~ 1)
    for side in ("l", "u"):
        lam, t = it["lam_" + side], it["t_" + side]
        act = rng.uniform(size=lam.size) < 0.5
        t[act] = 10.0 ** rng.uniform(-14, -10, act.sum())
        lam[~act] = 10.0 ** rng.uniform(-14, -10, (~act).sum())
    tau = 1e-12
    plain = O.newton_step(qp, it, tau)
    refined, kept = O.newton_step_refined(qp, it, tau, ir_max=4)
    r0 = _dense_ir_norm(dq, it, tau, plain)
    r1 = _dense_ir_norm(dq, it, tau, refined)
    assert kept >= 1 and r1 < 0.5 * r0, (r0, r1, kept)


def test_large_stage_stalls_without_refinement_and_converges_with_it():
    """Instance 1 of the large-stage batch: without refinement the
    stationarity residual grows again once the barrier weights span ~1e25 and
    the iteration ends on a too-short step; refining the
    prediction-centering-correction direction (up to 4 corrections) reaches
    KKT 1e-8."""
    qp = W.random_large_stage(1)
    plain = O.solve(qp, O.Arg.with_tol(1e-8))
    assert plain.status != O.SUCCESS
    assert plain.res[0] > 1e-6  # the stationarity residual is what stalls
    ref = O.solve(qp, O.Arg.with_tol(1e-8, ir_max=4))
    assert ref.status == O.SUCCESS, (ref.status, ref.res)
    assert ref.ir_steps > 0
    assert ref.iters <= 20
    # independent check of the returned point: dense residual of
    # eq:alg:pdipm:delta, stacked as the definition states
    dq = DenseQp(qp)
    rg, rb, rd, rm = dq.residual(ref.sol)
    kkt = max(np.max(np.abs(rg)), np.max(np.abs(rb)), np.max(np.abs(rd)), np.max(np.abs(rm)))
    assert kkt <= 1e-8, kkt


def test_refinement_refused_with_slacks_or_absolute_form():
    qp = W.mass_spring_chain8_soft(0)
    with pytest.raises(ValueError):
        O.solve(qp, O.Arg.with_tol(1e-8, ir_max=2))
    with pytest.raises(ValueError):
        O.solve(W.mass_spring_chain4(1), O.Arg.with_tol(1e-8, ir_max=2, abs_form=1))
