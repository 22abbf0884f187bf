"""Pins of the CPU oracle against definitions it does not share code with.

Each test names the passage it checks.  A plausible mistake in the oracle
(dropped term, wrong sign or index, transposed operand) makes one of them
fail: the residual and the Newton step are compared with dense evaluations
of eq:alg:pdipm:delta; the IPM's converged point with brute-force active-set
enumeration, the textbook LQR recursion and the DARE; plus the invariants of
the KKT conditions eq:alg:pdipm:kkt.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_02547_amd import workloads as W
from dense_ref import DenseQp, lqr_finite_horizon, dare_gain, random_interior_iterate

FLAT = ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u")


def _cmp(a, b, tol, what=""):
    for k in FLAT:
        x, y = np.asarray(a[k]), np.asarray(b[k])
        assert x.shape == y.shape, (what, k, x.shape, y.shape)
        if x.size:
            err = np.max(np.abs(x - y)) / max(1.0, np.max(np.abs(y)))
            assert err <= tol, (what, k, err)


def _tiny(seed, **kw):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(1, 5))
    return W.random_tiny(rng, N, **kw), rng


# ---------------------------------------------------------------------------
# Generators (Section 5.1 model; random stable systems)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("M,dt", [(4, 0.5), (8, 0.2)])
def test_mass_spring_discretisation(M, dt):
    import scipy.integrate
    A, B, Ac, Bc = W.mass_spring_model(M, dt)
    # undamped chain: every eigenvalue of A on the unit circle
    assert np.allclose(np.abs(np.linalg.eigvals(A)), 1.0, atol=1e-10)
    # B = int_0^dt expm(Ac s) Bc ds
    Bq, _ = scipy.integrate.quad_vec(lambda s: __import__("scipy.linalg").linalg.expm(Ac * s) @ Bc, 0.0, dt,
                                     epsabs=1e-13, epsrel=1e-13)
    assert np.allclose(B, Bq, atol=1e-11)
    assert A.shape == (2 * M, 2 * M) and B.shape == (2 * M, M - 1)


def test_random_stable_radius_and_feasible_rollout():
    for i in range(5):
        qp = W.random_uneven(i)
        A = qp.A[0]
        assert abs(np.max(np.abs(np.linalg.eigvals(A))) - 0.95) < 1e-10
        x = qp.meta["x0"].copy()
        for n in range(qp.N):
            x = A @ x
            assert np.all(np.abs(x) <= qp.ubx[n + 1] + 1e-12)
        assert 4 <= qp.nx[0] <= 48 and 1 <= qp.nu[0] <= 16 and 10 <= qp.N <= 100


def test_workload_shapes():
    qp = W.mass_spring_chain4(1)
    assert qp.N == 10 and qp.nx[0] == 8 and qp.nu[0] == 3 and qp.nu[10] == 0
    assert qp.nbx[0] == 8 and np.array_equal(qp.lbx[0], qp.ubx[0])
    assert qp.nbx[1] == 4 and qp.nbu[0] == 3
    qp = W.mass_spring_chain8(7)
    assert qp.N == 30 and qp.nx[5] == 16 and qp.nu[5] == 7
    assert np.all(np.abs(qp.meta["x0"]) <= 2.0)


# ---------------------------------------------------------------------------
# Residual function and Newton step, eq:alg:pdipm:delta
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_residual_matches_dense_definition(seed):
    qp, rng = _tiny(seed, ng_max=2)
    dq = DenseQp(qp)
    it = random_interior_iterate(qp, rng)
    parts, norms, mu = O.residuals(qp, it)
    rg, rb, rd, rm = dq.residual(it)
    ru, rx = dq.ux_from(rg)
    m = dq.m
    assert np.allclose(parts["u"], ru, atol=1e-12)
    assert np.allclose(parts["x"], rx, atol=1e-12)
    assert np.allclose(parts["pi"], rb, atol=1e-12)
    assert np.allclose(parts["lam_l"], rd[:m], atol=1e-12)
    assert np.allclose(parts["lam_u"], rd[m:], atol=1e-12)
    assert np.allclose(parts["t_l"], rm[:m], atol=1e-12)
    assert np.isclose(norms[0], np.max(np.abs(rg)), atol=1e-12)
    if m:
        assert np.isclose(mu, np.sum(rm) / (2 * m), atol=1e-12)


@pytest.mark.parametrize("seed", range(40))
def test_newton_step_matches_dense_lu(seed):
    """Classical Riccati step == dense LU of the full 4-block matrix of
    eq:alg:pdipm:delta, on tiny instances with stage-varying sizes."""
    mode = ["box", "free", "eliminated"][seed % 3]
    qp, rng = _tiny(seed, ng_max=2, x0_mode=mode)
    dq = DenseQp(qp)
    it = random_interior_iterate(qp, rng)
    tau = float(rng.uniform(0.0, 0.5))
    ref = dq.newton_step(it, tau)
    got = O.newton_step(qp, it, tau)
    _cmp(got, ref, 1e-9, f"seed {seed}")
    # the reduced system eq:alg:kkt gives the same step
    _cmp(dq.reduced_step(it, tau), ref, 1e-9, "reduced")


def test_newton_step_with_regularization_differs_by_design():
    qp, rng = _tiny(3, ng_max=1)
    it = random_interior_iterate(qp, rng)
    a = O.newton_step(qp, it, 0.1, reg=0.0)
    b = O.newton_step(qp, it, 0.1, reg=1e-2)
    assert np.max(np.abs(a["x"] - b["x"])) > 1e-8


@pytest.mark.parametrize("seed", range(6))
def test_ir_residual_zero_at_exact_step(seed):
    """Section 3.4: the iterative-refinement residual K*step + r vanishes at
    the exact step and equals K*(step error) otherwise."""
    qp, rng = _tiny(seed, ng_max=1)
    dq = DenseQp(qp)
    it = random_interior_iterate(qp, rng)
    step = dq.newton_step(it, 0.05)
    rg, rb, rd, rm = dq.residual(it, 0.05)
    m = dq.m
    ru, rx = dq.ux_from(rg)
    rhs = dict(u=ru, x=rx, pi=rb, lam_l=rd[:m], lam_u=rd[m:], t_l=rm[:m], t_u=rm[m:])
    r0 = O.ir_residual(qp, it, step, rhs)
    for k in FLAT:
        assert np.max(np.abs(r0[k]), initial=0) < 1e-9
    pert = {k: np.asarray(v) + 1e-3 * rng.standard_normal(np.shape(v)) for k, v in step.items()}
    r1 = O.ir_residual(qp, it, pert, rhs)
    K = dq.kkt_matrix(it)
    y, pi, lam, t = dq.stack({**pert})
    ys, pis, lams, ts = dq.stack({**step})
    full = K @ np.concatenate([y - ys, pi - pis, lam - lams, t - ts])
    nv, ne = dq.nv, dq.neq
    fu, fx = dq.ux_from(full[:nv])
    assert np.allclose(r1["u"], fu, atol=1e-10) and np.allclose(r1["x"], fx, atol=1e-10)
    assert np.allclose(r1["pi"], full[nv:nv + ne], atol=1e-10)


# ---------------------------------------------------------------------------
# Unconstrained special case: finite-horizon LQR and the DARE
# ---------------------------------------------------------------------------

def _lqr_qp(A, B, Q, R, QN, N, x0):
    nx, nu = B.shape
    nxl = [0] + [nx] * N
    nul = [nu] * N + [0]
    Al = [np.zeros((nx, 0))] + [A] * (N - 1)
    bl = [A @ x0] + [np.zeros(nx)] * (N - 1)
    Ql = [np.zeros((0, 0))] + [Q] * (N - 1) + [QN]
    Sl = [np.zeros((nu, 0))] + [np.zeros((nu, nx))] * (N - 1) + [np.zeros((0, nx))]
    Rl = [R] * N + [np.zeros((0, 0))]
    ql = [np.zeros(0)] + [np.zeros(nx)] * N
    rl = [np.zeros(nu)] * N + [np.zeros(0)]
    return W.assemble(N, nxl, nul, Al, [B] * N, bl, Ql, Sl, Rl, ql, rl)


@pytest.mark.parametrize("seed", range(4))
def test_unconstrained_matches_textbook_lqr(seed):
    rng = np.random.default_rng(100 + seed)
    nx, nu, N = 4, 2, 8
    A = rng.standard_normal((nx, nx)) * 0.6
    B = rng.standard_normal((nx, nu))
    Q = np.diag(rng.uniform(0.5, 2, nx)); R = np.diag(rng.uniform(0.5, 2, nu))
    QN = 2.0 * Q
    x0 = rng.standard_normal(nx)
    qp = _lqr_qp(A, B, Q, R, QN, N, x0)
    res = O.solve(qp, O.Arg.with_tol(1e-12))
    assert res.status == O.SUCCESS and res.iters == 1  # one exact Newton step from zero
    us, xs, _ = lqr_finite_horizon(A, B, Q, R, QN, N, x0)
    assert np.allclose(res.sol["u"], np.concatenate(us), atol=1e-10)
    assert np.allclose(res.sol["x"], np.concatenate(xs[1:]), atol=1e-10)


def test_unconstrained_with_dare_terminal_is_stationary_gain():
    rng = np.random.default_rng(7)
    W_, _ = W.mass_spring_model(3, 0.4)[:2], None
    A, B, _, _ = W.mass_spring_model(3, 0.4)
    nx, nu = B.shape
    Q, R = np.eye(nx), 0.5 * np.eye(nu)
    P, K = dare_gain(A, B, Q, R)
    x0 = rng.standard_normal(nx)
    N = 12
    qp = _lqr_qp(A, B, Q, R, P, N, x0)
    res = O.solve(qp, O.Arg.with_tol(1e-12))
    u = res.sol["u"].reshape(N, nu)
    x = np.concatenate([x0, res.sol["x"]]).reshape(N + 1, nx)
    for n in range(N):
        assert np.allclose(u[n], -K @ x[n], atol=1e-9)


# ---------------------------------------------------------------------------
# The exact result: brute-force active sets on tiny QPs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(10))
def test_ipm_reaches_brute_force_minimiser(seed):
    rng = np.random.default_rng(1000 + seed)
    while True:
        qp = W.random_tiny(rng, int(rng.integers(1, 3)), nx_range=(1, 3), nu_range=(1, 2),
                           nb_frac=0.6, ng_max=1, x0_mode=["box", "eliminated"][seed % 2])
        dq = DenseQp(qp)
        nfree = int(np.sum(~np.isclose(dq.lo, dq.hi, rtol=0, atol=0)))
        if 1 <= nfree <= 8:
            break
    cands = dq.brute_force()
    if not cands:
        pytest.skip("random tiny QP infeasible")
    ystar = cands[0]
    for y in cands[1:]:
        assert np.allclose(y, ystar, atol=1e-8)
    res = O.solve(qp, O.Arg.with_tol(1e-10))
    assert res.status == O.SUCCESS, res
    y = dq.y_from(res.sol["u"], res.sol["x"])
    assert np.max(np.abs(y - ystar)) / max(1.0, np.max(np.abs(ystar))) < 1e-7


# ---------------------------------------------------------------------------
# Invariants of eq:alg:pdipm:kkt at the returned point
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def chain4():
    qp = W.mass_spring_chain4(1)
    return qp, O.solve(qp, O.Arg.with_tol(1e-10))


def test_chain4_converges_and_is_kkt_point(chain4):
    qp, res = chain4
    assert res.status == O.SUCCESS
    assert np.max(res.res) <= 1e-10
    s = res.sol
    for k in ("lam_l", "lam_u", "t_l", "t_u"):
        assert np.all(s[k] > 0)
    dq = DenseQp(qp)
    rg, rb, rd, rm = dq.residual(s)
    assert max(np.abs(rg).max(), np.abs(rb).max(), np.abs(rd).max(), np.abs(rm).max()) <= 1e-10


def test_duality_gap_equals_lam_t(chain4):
    """primal - dual objective = lam't at a point with r_g = r_b = r_d = 0."""
    qp, res = chain4
    dq = DenseQp(qp)
    y, pi, lam, t = dq.stack(res.sol)
    primal = 0.5 * y @ dq.H @ y + dq.g @ y
    dual = -0.5 * y @ dq.H @ y + dq.beq @ pi + dq.d @ lam
    assert abs((primal - dual) - lam @ t) < 1e-8


def test_odd_symmetry_in_x0():
    x0 = np.random.default_rng(3).uniform(-1, 1, 8)
    a = O.solve(W.mass_spring(4, 10, 0.5, 1.0, x0), O.Arg.with_tol(1e-11))
    b = O.solve(W.mass_spring(4, 10, 0.5, 1.0, -x0), O.Arg.with_tol(1e-11))
    assert np.allclose(a.sol["u"], -b.sol["u"], atol=1e-8)
    assert np.allclose(a.sol["x"], -b.sol["x"], atol=1e-8)


def test_zero_x0_gives_zero_solution():
    res = O.solve(W.mass_spring(4, 10, 0.5, 1.0, np.zeros(8)), O.Arg.with_tol(1e-11))
    assert res.status == O.SUCCESS
    assert np.max(np.abs(res.sol["u"])) < 1e-9 and np.max(np.abs(res.sol["x"])) < 1e-9


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_x0_box_and_eliminated_forms_agree(seed):
    qp = W.mass_spring_chain4(seed)
    qe = W.eliminate_x0(qp)
    a = O.solve(qp, O.Arg.with_tol(1e-11))
    b = O.solve(qe, O.Arg.with_tol(1e-11))
    assert a.status == O.SUCCESS and b.status == O.SUCCESS
    assert np.allclose(a.sol["u"], b.sol["u"], atol=1e-8)
    assert np.allclose(a.sol["x"][8:], b.sol["x"], atol=1e-8)


def test_status_paths():
    qp = W.mass_spring_chain4(1)
    r = O.solve(qp, O.Arg.with_tol(1e-10, iter_max=1))
    assert r.status == O.MAX_ITER and r.iters == 1
    bad = qp.copy()
    bad.Q[3] = bad.Q[3].copy(); bad.Q[3][0, 0] = np.nan
    r = O.solve(bad)
    assert r.status == O.NAN
    bad = qp.copy()
    bad.lbu[2] = bad.lbu[2].copy(); bad.lbu[2][0] = 1.0  # lo > hi
    with pytest.raises(ValueError):
        O.solve(bad)
