"""Seeded synthetic OCP-QP workloads.

This module only builds problem data: it holds none of the solver's
arithmetic.  Both the HIP path and the CPU oracle read the arrays it
produces, so random-number details cannot break parity between them.

Problem form (Section 2.2, the OCP QP): stages n = 0..N, stage variable
z_n = [u_n; x_n], dynamics x_{n+1} = A_n x_n + B_n u_n + b_n, stage cost
1/2 z'[[R, S], [S', Q]] z + [r; q]'z with S of shape nu x nx, box
constraints on selected components of u_n and x_n given as index lists, and
two-sided general constraints lg <= D_n u_n + C_n x_n <= ug.  The initial
state is fixed by a box with equal lower and upper limits (Section 2.2, the
note on equality constraints other than the dynamics).

Workload families:
  * the linear mass-spring chain (Section 5.1): M masses, nx = 2M,
    nu = M - 1, unit masses and springs, walls at both ends, zero-order-hold
    discretisation by matrix exponential;
  * random stable systems: A Gaussian rescaled to spectral radius 0.95,
    B Gaussian / sqrt(nx), diagonal Q and R, boxes on all u and x, and
    optionally Gaussian general constraints on u.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg


@dataclass
class OcpQp:
    """One OCP QP in column-major-friendly numpy arrays (all float64).

    Lists indexed by stage.  Dynamics lists (A, B, b) have N entries; all
    other lists have N + 1 entries.  Empty constraints use arrays of length 0.
    """

    N: int
    nx: List[int]
    nu: List[int]
    A: List[np.ndarray]
    B: List[np.ndarray]
    b: List[np.ndarray]
    Q: List[np.ndarray]
    S: List[np.ndarray]
    R: List[np.ndarray]
    q: List[np.ndarray]
    r: List[np.ndarray]
    idxbu: List[np.ndarray]
    lbu: List[np.ndarray]
    ubu: List[np.ndarray]
    idxbx: List[np.ndarray]
    lbx: List[np.ndarray]
    ubx: List[np.ndarray]
    D: List[np.ndarray]
    C: List[np.ndarray]
    lg: List[np.ndarray]
    ug: List[np.ndarray]
    meta: dict = field(default_factory=dict)
    # Soft constraints (Section 2.2, the slack variables), or None: per
    # stage, the rows relaxed by a slack pair (indices into the stage's rows
    # [box u, box x, general]; the lower row gains +s^l, the upper row -s^u),
    # the slacks' diagonal Hessians Zl, Zu, gradients zl, zu and lower
    # bounds lls, lus (s^l >= lls, s^u >= lus).
    idxs: Optional[List[np.ndarray]] = None
    Zl: Optional[List[np.ndarray]] = None
    Zu: Optional[List[np.ndarray]] = None
    zl: Optional[List[np.ndarray]] = None
    zu: Optional[List[np.ndarray]] = None
    lls: Optional[List[np.ndarray]] = None
    lus: Optional[List[np.ndarray]] = None

    @property
    def nbu(self):
        return [len(i) for i in self.idxbu]

    @property
    def nbx(self):
        return [len(i) for i in self.idxbx]

    @property
    def ng(self):
        return [d.shape[0] for d in self.D]

    @property
    def ns(self):
        return [len(i) for i in self.idxs] if self.idxs is not None else [0] * (self.N + 1)

    def n_constraints(self) -> int:
        """Number of two-sided constraint rows (each counted once)."""
        return sum(self.nbu) + sum(self.nbx) + sum(self.ng)

    def copy(self) -> "OcpQp":
        cp = lambda L: [np.array(a, copy=True) for a in L]
        return OcpQp(self.N, list(self.nx), list(self.nu), cp(self.A), cp(self.B), cp(self.b),
                     cp(self.Q), cp(self.S), cp(self.R), cp(self.q), cp(self.r),
                     cp(self.idxbu), cp(self.lbu), cp(self.ubu), cp(self.idxbx), cp(self.lbx),
                     cp(self.ubx), cp(self.D), cp(self.C), cp(self.lg), cp(self.ug), dict(self.meta),
                     *[None if getattr(self, k) is None else cp(getattr(self, k)) for k in SOFT_FIELDS])


SOFT_FIELDS = ("idxs", "Zl", "Zu", "zl", "zu", "lls", "lus")


def soften(qp: OcpQp, rows, Zl, Zu, zl, zu, lls=0.0, lus=0.0) -> OcpQp:
    """A copy of `qp` with the constraint rows rows(n, qp) of each stage
    (indices into [box u, box x, general]) made soft, each slack pair with the
    scalar penalty weights Zl, Zu (quadratic), zl, zu (linear) and lower
    bounds lls, lus (Section 2.2)."""
    out = qp.copy()
    idxs = [np.asarray(rows(n, qp), dtype=np.int32) for n in range(qp.N + 1)]
    out.idxs = idxs
    for k, v in (("Zl", Zl), ("Zu", Zu), ("zl", zl), ("zu", zu), ("lls", lls), ("lus", lus)):
        setattr(out, k, [np.full(len(i), float(v)) for i in idxs])
    return out


def state_box_rows(n, qp):
    """The rows of stage n's state boxes, stage 0 excluded (x_0 stays fixed)."""
    if n == 0:
        return []
    nbu = len(qp.idxbu[n])
    return list(range(nbu, nbu + len(qp.idxbx[n])))


def _empty_i():
    return np.zeros(0, dtype=np.int32)


def _empty_f():
    return np.zeros(0, dtype=np.float64)


def assemble(N, nx, nu, A, B, b, Q, S, R, q, r, *, boxu=None, boxx=None, gen=None) -> OcpQp:
    """Build an OcpQp from per-stage lists; boxu/boxx/gen are per-stage tuples
    (idx, lo, hi) / (D, C, lo, hi) or None for no constraint at that stage."""
    idxbu, lbu, ubu, idxbx, lbx, ubx, D, C, lg, ug = ([] for _ in range(10))
    for n in range(N + 1):
        bu = boxu[n] if boxu is not None else None
        if bu is None:
            idxbu.append(_empty_i()); lbu.append(_empty_f()); ubu.append(_empty_f())
        else:
            idxbu.append(np.asarray(bu[0], dtype=np.int32))
            lbu.append(np.asarray(bu[1], dtype=np.float64))
            ubu.append(np.asarray(bu[2], dtype=np.float64))
        bx = boxx[n] if boxx is not None else None
        if bx is None:
            idxbx.append(_empty_i()); lbx.append(_empty_f()); ubx.append(_empty_f())
        else:
            idxbx.append(np.asarray(bx[0], dtype=np.int32))
            lbx.append(np.asarray(bx[1], dtype=np.float64))
            ubx.append(np.asarray(bx[2], dtype=np.float64))
        gg = gen[n] if gen is not None else None
        if gg is None:
            D.append(np.zeros((0, nu[n]))); C.append(np.zeros((0, nx[n])))
            lg.append(_empty_f()); ug.append(_empty_f())
        else:
            D.append(np.asarray(gg[0], dtype=np.float64)); C.append(np.asarray(gg[1], dtype=np.float64))
            lg.append(np.asarray(gg[2], dtype=np.float64)); ug.append(np.asarray(gg[3], dtype=np.float64))
    f = lambda L: [np.asarray(a, dtype=np.float64) for a in L]
    return OcpQp(N, list(nx), list(nu), f(A), f(B), f(b), f(Q), f(S), f(R), f(q), f(r),
                 idxbu, lbu, ubu, idxbx, lbx, ubx, D, C, lg, ug)


# ---------------------------------------------------------------------------
# Linear mass-spring chain (Section 5.1)
# ---------------------------------------------------------------------------

def mass_spring_model(M: int, dt: float):
    """Zero-order-hold discretisation of the chain of M unit masses joined by
    M + 1 unit springs (walls at both ends); a force acts on each of the first
    M - 1 masses.  State [p_1..p_M, v_1..v_M].  Returns (A, B, A_c, B_c)."""
    K = 2.0 * np.eye(M) - np.eye(M, k=1) - np.eye(M, k=-1)
    Ac = np.zeros((2 * M, 2 * M))
    Ac[:M, M:] = np.eye(M)
    Ac[M:, :M] = -K
    Bc = np.zeros((2 * M, M - 1))
    Bc[M:M + M - 1, :] = np.eye(M - 1)
    aug = np.zeros((3 * M - 1, 3 * M - 1))
    aug[:2 * M, :2 * M] = Ac
    aug[:2 * M, 2 * M:] = Bc
    E = scipy.linalg.expm(aug * dt)
    return E[:2 * M, :2 * M].copy(), E[:2 * M, 2 * M:].copy(), Ac, Bc


def mass_spring(M: int, N: int, dt: float, r_weight: float, x0: np.ndarray, *,
                u_max: float = 0.5, x_max: float = 4.0, box_all_states: bool = False) -> OcpQp:
    """Mass-spring OCP QP: Q = I, R = r_weight I, terminal Q_N = Q, box |u| <= u_max
    on all inputs, |x| <= x_max on the positions (or on every state with
    box_all_states, the count nb = 3M - 1 of Section 5.1), x_0 fixed by an
    equal-limit box."""
    A, B, _, _ = mass_spring_model(M, dt)
    nx_, nu_ = 2 * M, M - 1
    nx = [nx_] * (N + 1)
    nu = [nu_] * N + [0]
    Al = [A] * N
    Bl = [B] * N
    bl = [np.zeros(nx_)] * N
    Q = [np.eye(nx_)] * (N + 1)
    S = [np.zeros((nu_, nx_))] * N + [np.zeros((0, nx_))]
    R = [r_weight * np.eye(nu_)] * N + [np.zeros((0, 0))]
    q = [np.zeros(nx_)] * (N + 1)
    r = [np.zeros(nu_)] * N + [np.zeros(0)]
    iu = np.arange(nu_)
    boxu = [(iu, -u_max * np.ones(nu_), u_max * np.ones(nu_))] * N + [None]
    ix = np.arange(nx_) if box_all_states else np.arange(M)
    boxx = [(np.arange(nx_), x0.copy(), x0.copy())]
    boxx += [(ix, -x_max * np.ones(len(ix)), x_max * np.ones(len(ix)))] * N
    qp = assemble(N, nx, nu, Al, Bl, bl, Q, S, R, q, r, boxu=boxu, boxx=boxx)
    qp.meta.update(family="mass_spring", M=M, dt=dt, x0=x0.copy())
    return qp


def mass_spring_chain4(seed: int = 1) -> OcpQp:
    """Single QP: 4 masses (nx=8, nu=3), dt=0.5, N=10, Q=I, R=I, box |u|<=0.5,
    |x_pos|<=4, x0 ~ U[-1,1]^8 from the seed."""
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-1.0, 1.0, 8)
    qp = mass_spring(4, 10, 0.5, 1.0, x0)
    qp.meta["seed"] = seed
    return qp


def mass_spring_chain8(i: int) -> OcpQp:
    """Instance i of the same-size batch: 8 masses (nx=16, nu=7), N=30,
    dt=0.2, Q=I, R=0.1 I, same boxes, x0 ~ U[-2,2]^16."""
    rng = np.random.default_rng(np.random.SeedSequence([2, i]))
    x0 = rng.uniform(-2.0, 2.0, 16)
    qp = mass_spring(8, 30, 0.2, 0.1, x0)
    qp.meta["instance"] = i
    return qp


# ---------------------------------------------------------------------------
# Random stable systems
# ---------------------------------------------------------------------------

def _zero_input_rollout_ok(A, x0, N, hx):
    x = x0.copy()
    for _ in range(N):
        x = A @ x
        if np.any(np.abs(x) > hx):
            return False
    return True


def random_stable(rng: np.random.Generator, nx: int, nu: int, N: int, ng: int = 0,
                  max_redraw: int = 10000, redraw: bool = True) -> OcpQp:
    """Random time-invariant OCP QP with a fixed draw order:
    G ~ N(0,1) (nx x nx), A = 0.95 G / rho(G); B ~ N(0,1)/sqrt(nx);
    Q = diag U[0.1,10]; R = diag U[0.1,1]; S = 0, q = r = b = 0;
    box half-widths U[0.5,2] on u and U[2,5] on x (all components boxed);
    if ng > 0: D ~ N(0,1) (ng x nu), C = 0, bounds +-U[1,3] at stages 0..N-1;
    x0 ~ N(0,1), redrawn from the same stream until the zero-input rollout
    stays inside every state box (so u = 0 is a feasible point); with
    redraw=False the first draw is kept (the problem may be infeasible)."""
    Gm = rng.standard_normal((nx, nx))
    rho = np.max(np.abs(np.linalg.eigvals(Gm)))
    A = Gm * (0.95 / rho)
    B = rng.standard_normal((nx, nu)) / np.sqrt(nx)
    Qd = rng.uniform(0.1, 10.0, nx)
    Rd = rng.uniform(0.1, 1.0, nu)
    hu = rng.uniform(0.5, 2.0, nu)
    hx = rng.uniform(2.0, 5.0, nx)
    if ng > 0:
        Dm = rng.standard_normal((ng, nu))
        hg = rng.uniform(1.0, 3.0, ng)
    redraws = 0
    while True:
        x0 = rng.standard_normal(nx)
        if not redraw or _zero_input_rollout_ok(A, x0, N, hx):
            break
        redraws += 1
        if redraws >= max_redraw:
            raise RuntimeError("no x0 with a feasible zero-input rollout found")
    nxl = [nx] * (N + 1)
    nul = [nu] * N + [0]
    Q = np.diag(Qd)
    R = np.diag(Rd)
    iu, ix = np.arange(nu), np.arange(nx)
    boxu = [(iu, -hu, hu)] * N + [None]
    boxx = [(ix, x0.copy(), x0.copy())] + [(ix, -hx, hx)] * N
    gen = None
    if ng > 0:
        gen = [(Dm, np.zeros((ng, nx)), -hg, hg)] * N + [None]
    qp = assemble(N, nxl, nul, [A] * N, [B] * N, [np.zeros(nx)] * N, [Q] * (N + 1),
                  [np.zeros((nu, nx))] * N + [np.zeros((0, nx))], [R] * N + [np.zeros((0, 0))],
                  [np.zeros(nx)] * (N + 1), [np.zeros(nu)] * N + [np.zeros(0)],
                  boxu=boxu, boxx=boxx, gen=gen)
    qp.meta.update(family="random_stable", x0=x0.copy(), redraws=redraws)
    return qp


def random_uneven(i: int) -> OcpQp:
    """Instance i of the uneven batch: nx ~ U{4..48}, nu ~ U{1..16},
    N ~ U{10..100}, then random_stable."""
    rng = np.random.default_rng(np.random.SeedSequence([3, i]))
    nx = int(rng.integers(4, 49))
    nu = int(rng.integers(1, 17))
    N = int(rng.integers(10, 101))
    qp = random_stable(rng, nx, nu, N)
    qp.meta["instance"] = i
    return qp


# Soft-constraint workloads (Section 2.2): every state box after stage 0
# softened with an L2 weight of 1 and an L1 weight of 10 per slack.
SOFT_Z, SOFT_z = 1.0, 10.0


def mass_spring_chain8_soft(i: int) -> OcpQp:
    """Instance i of the 8-mass batch with soft position boxes (every
    instance feasible, including those whose hard boxes are not)."""
    return soften(mass_spring_chain8(i), state_box_rows, SOFT_Z, SOFT_Z, SOFT_z, SOFT_z)


def random_uneven_soft(i: int) -> OcpQp:
    """Instance i of the uneven batch with its first x0 draw (no redraw for
    a feasible zero-input rollout) and soft state boxes."""
    rng = np.random.default_rng(np.random.SeedSequence([3, i]))
    nx = int(rng.integers(4, 49))
    nu = int(rng.integers(1, 17))
    N = int(rng.integers(10, 101))
    qp = random_stable(rng, nx, nu, N, redraw=False)
    qp.meta["instance"] = i
    return soften(qp, state_box_rows, SOFT_Z, SOFT_Z, SOFT_z, SOFT_z)


def soften_random(qp: OcpQp, rng: np.random.Generator, frac: float = 0.6) -> OcpQp:
    """A random subset (about frac) of each stage's rows made soft, stage 0's
    state box kept hard, with random weights Zl, Zu ~ U[0.1, 3], zl, zu ~
    U[0, 2] and slack bounds lls, lus ~ U[0, 0.2]."""
    out = qp.copy()
    idxs, vals = [], {k: [] for k in ("Zl", "Zu", "zl", "zu", "lls", "lus")}
    for n in range(qp.N + 1):
        nc = qp.nbu[n] + qp.nbx[n] + qp.ng[n]
        cand = list(range(nc))
        if n == 0:
            nbu = qp.nbu[0]
            cand = [k for k in cand if not (nbu <= k < nbu + qp.nbx[0])]
        pick = [k for k in cand if rng.uniform() < frac]
        rng.shuffle(pick)
        idxs.append(np.asarray(pick, dtype=np.int32))
        m = len(pick)
        vals["Zl"].append(rng.uniform(0.1, 3.0, m)); vals["Zu"].append(rng.uniform(0.1, 3.0, m))
        vals["zl"].append(rng.uniform(0.0, 2.0, m)); vals["zu"].append(rng.uniform(0.0, 2.0, m))
        vals["lls"].append(rng.uniform(0.0, 0.2, m)); vals["lus"].append(rng.uniform(0.0, 0.2, m))
    out.idxs = idxs
    for k, v in vals.items():
        setattr(out, k, v)
    return out


def random_large_stage(i: int) -> OcpQp:
    """Instance i of the large-stage batch: nx=128, nu=32, N=50, 32 general
    constraints on u per stage."""
    rng = np.random.default_rng(np.random.SeedSequence([5, i]))
    qp = random_stable(rng, 128, 32, 50, ng=32)
    qp.meta["instance"] = i
    return qp


def serving_stream(rate: float, duration: float, pool: int, seed: int = 4):
    """Poisson arrivals at `rate` per second over `duration` seconds
    (exponential inter-arrival times) and, per arrival, the index of the
    request it sends, drawn uniformly from a pool of `pool` pre-generated
    instances of the uneven distribution."""
    rng = np.random.default_rng(np.random.SeedSequence([4, seed]))
    t, times = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        times.append(t)
    idx = rng.integers(0, pool, size=len(times))
    return np.asarray(times), idx


def receding_step(qp: OcpQp, sol: dict):
    """The next problem of a receding-horizon loop on a chain QP (same stage
    sizes at stages 0..N-1, x_0 fixed by an equal-limit box) and its guess:
    x_0 <- x_1 of `sol`; the guess takes stage n + 1 of `sol` at stage n (the
    last stage repeated), multipliers and slacks pushed to at least 1.
    Data handling only."""
    N, nx, nu = qp.N, qp.nx[1], qp.nu[0]
    nxt = qp.copy()
    x1 = np.asarray(sol["x"][nx:2 * nx], dtype=np.float64)
    nxt.lbx[0], nxt.ubx[0] = x1.copy(), x1.copy()
    u = np.asarray(sol["u"]).reshape(N, nu)
    x = np.asarray(sol["x"]).reshape(N + 1, nx)
    pi = np.asarray(sol["pi"]).reshape(N, nx)
    guess = {"u": np.concatenate([u[1:], u[-1:]]).ravel(), "x": np.concatenate([x[1:], x[-1:]]).ravel(),
             "pi": np.concatenate([pi[1:], pi[-1:]]).ravel()}
    for k in ("lam_l", "lam_u", "t_l", "t_u"):
        guess[k] = np.maximum(np.asarray(sol[k], dtype=np.float64), 1.0)
    # slack blocks (soft constraints): kept in place like the row blocks
    for k in ("s_l", "s_u"):
        if k in sol:
            guess[k] = np.asarray(sol[k], dtype=np.float64).copy()
    for k in ("lam_sl", "lam_su", "t_sl", "t_su"):
        if k in sol:
            guess[k] = np.maximum(np.asarray(sol[k], dtype=np.float64), 1.0)
    return nxt, guess


def random_tiny(rng: np.random.Generator, N: int, nx_range=(1, 4), nu_range=(0, 3),
                nb_frac: float = 0.5, ng_max: int = 1, x0_mode: str = "box",
                time_varying: bool = True) -> OcpQp:
    """Small random OCP QP with stage-varying sizes and data, used for
    checks that need dense or brute-force references.  Q, R from random
    SPD matrices with a random coupling S small enough that the stage
    Hessian stays positive definite.  x0_mode: 'box' (x_0 fixed by an
    equal-limit box), 'free' (no constraint on x_0), or 'eliminated'
    (nx_0 = 0)."""
    nx = [int(rng.integers(nx_range[0], nx_range[1] + 1)) for _ in range(N + 1)]
    nu = [int(rng.integers(nu_range[0], nu_range[1] + 1)) for _ in range(N + 1)]
    if x0_mode == "eliminated":
        nx[0] = 0
        nu[0] = max(nu[0], 1)
    A, B, b, Q, S, R, q, r = ([] for _ in range(8))
    boxu, boxx, gen = [], [], []
    x0 = rng.standard_normal(nx[0])
    for n in range(N + 1):
        if n < N:
            A.append(rng.standard_normal((nx[n + 1], nx[n])) * 0.7)
            B.append(rng.standard_normal((nx[n + 1], nu[n])))
            b.append(rng.standard_normal(nx[n + 1]) * 0.3)
        nz = nx[n] + nu[n]
        Wm = rng.standard_normal((nz, nz))
        H = Wm @ Wm.T / max(nz, 1) + 0.5 * np.eye(nz)
        R.append(H[:nu[n], :nu[n]].copy())
        S.append(H[:nu[n], nu[n]:].copy())
        Q.append(H[nu[n]:, nu[n]:].copy())
        q.append(rng.standard_normal(nx[n]))
        r.append(rng.standard_normal(nu[n]))
        # boxes
        ku = [j for j in range(nu[n]) if rng.uniform() < nb_frac]
        if ku:
            lo = -rng.uniform(0.2, 1.5, len(ku)); hi = rng.uniform(0.2, 1.5, len(ku))
            boxu.append((np.array(ku), lo, hi))
        else:
            boxu.append(None)
        if n == 0 and x0_mode == "box" and nx[0] > 0:
            boxx.append((np.arange(nx[0]), x0.copy(), x0.copy()))
        else:
            kx = [j for j in range(nx[n]) if rng.uniform() < nb_frac]
            if kx:
                lo = -rng.uniform(0.5, 3.0, len(kx)); hi = rng.uniform(0.5, 3.0, len(kx))
                boxx.append((np.array(kx), lo, hi))
            else:
                boxx.append(None)
        ngn = int(rng.integers(0, ng_max + 1)) if nz > 0 else 0
        if ngn > 0:
            Dm = rng.standard_normal((ngn, nu[n])); Cm = rng.standard_normal((ngn, nx[n]))
            lo = -rng.uniform(0.5, 2.0, ngn); hi = rng.uniform(0.5, 2.0, ngn)
            gen.append((Dm, Cm, lo, hi))
        else:
            gen.append(None)
    qp = assemble(N, nx, nu, A, B, b, Q, S, R, q, r, boxu=boxu, boxx=boxx, gen=gen)
    qp.meta.update(family="tiny", x0=x0)
    return qp


def eliminate_x0(qp: OcpQp) -> OcpQp:
    """Rewrite a QP whose x_0 is fixed by an equal-limit box on every state
    into the form with nx_0 = 0: b_0 <- A_0 x0 + b_0, r_0 <- r_0 + S_0 x0,
    the stage-0 general rows shift their bounds by C_0 x0.  Data rewriting
    only (the two forms have the same minimiser in u and x_1..x_N)."""
    x0 = np.zeros(qp.nx[0])
    assert len(qp.idxbx[0]) == qp.nx[0] and np.allclose(qp.lbx[0], qp.ubx[0])
    x0[qp.idxbx[0]] = qp.lbx[0]
    out = qp.copy()
    out.nx[0] = 0
    out.b[0] = qp.A[0] @ x0 + qp.b[0]
    out.A[0] = np.zeros((qp.nx[1], 0))
    out.r[0] = qp.r[0] + qp.S[0] @ x0
    out.S[0] = np.zeros((qp.nu[0], 0))
    out.Q[0] = np.zeros((0, 0))
    out.q[0] = np.zeros(0)
    out.idxbx[0] = _empty_i(); out.lbx[0] = _empty_f(); out.ubx[0] = _empty_f()
    if qp.D[0].shape[0] > 0:
        shift = qp.C[0] @ x0
        out.lg[0] = qp.lg[0] - shift
        out.ug[0] = qp.ug[0] - shift
        out.C[0] = np.zeros((qp.D[0].shape[0], 0))
    else:
        out.C[0] = np.zeros((0, 0))
    return out
