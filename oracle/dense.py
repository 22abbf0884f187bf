"""Full condensing of an OCP QP into the dense QP type and an IPM for it.

TEST INFRASTRUCTURE ONLY: the test suite uses it; the GPU path never does,
and nothing here imports the GPU package.

Condensing (Section 3.5) eliminates every state but the one at stage 0: the
dense QP of Section 2.1 has the variables v = [u_0; ...; u_N; x_0], no
equality constraints (the dynamics are substituted), and two-sided rows.
What is computed follows from that definition, with dense numpy algebra:

* states by forward substitution of the dynamics: x_n = X_n v + c_n with
  X_0 = [0 I], c_0 = 0, X_{n+1} = A_n X_n + B_n S_n, c_{n+1} = A_n c_n + b_n
  (S_n selects u_n from v);
* cost: with z_n = E_n v + e_n, E_n = [S_n; X_n], e_n = [0; c_n],
  H = sum_n E_n' H_n E_n and g = sum_n E_n' (H_n e_n + g_n), where
  H_n = [[R, S], [S', Q]] and g_n = [r; q] (stage N: Q_N, q_N only); the
  constant of the condensed cost is dropped (it does not move the minimiser);
* rows: input boxes and the box of x_0 are boxes on v; state boxes of
  stages 1..N become general rows X_n[i, :] with bounds shifted by c_n[i];
  general rows D_n u_n + C_n x_n become D_n S_n + C_n X_n with bounds shifted
  by C_n c_n.

The IPM is the method of Section 4 on this QP (Mehrotra predictor-corrector
in the delta formulation, eq:alg:pdipm:delta, with the conditional
corrector), with the Newton system reduced to the normal equations of v:
since there are no equality constraints, the KKT matrix of eq:alg:kkt is
H + A' W A (A: every row, boxes as unit rows; W = diag(lam / t) summed over
the two sides of each row), factored by one dense Cholesky factorization
(numpy) per iteration, the solver Section 3.3 names for condensed QPs.  The
same constants and rules as the OCP oracle: cold start v = 0, t = max(A v -
lo, 1) and max(hi - A v, 1), lam = 1; sigma = (mu_aff / mu)^3; corrector
rejected when the duality measure after its step exceeds corr_ratio * mu_aff;
step alpha = min(1, gamma alpha_max); clamps lam, t >= 1e-16; exit when the
four residual inf-norms are within tolerance.
"""
from __future__ import annotations

from types import SimpleNamespace
from typing import Dict

import numpy as np
import scipy.linalg as sla


def _stage_H(qp, n):
    nu, nx = qp.nu[n], qp.nx[n]
    H = np.zeros((nu + nx, nu + nx))
    H[:nu, :nu] = np.asarray(qp.R[n]).reshape(nu, nu)
    H[:nu, nu:] = np.asarray(qp.S[n]).reshape(nu, nx)
    H[nu:, :nu] = np.asarray(qp.S[n]).reshape(nu, nx).T
    H[nu:, nu:] = np.asarray(qp.Q[n]).reshape(nx, nx)
    return H


def state_maps(qp):
    """X_n (nx_n x nv) and c_n with x_n = X_n v + c_n, n = 0..N, and the
    offsets of the inputs u_n in v."""
    N = qp.N
    nus = [qp.nu[n] for n in range(N + 1)]
    off = np.concatenate([[0], np.cumsum(nus)]).astype(int)
    nU = int(off[-1])
    nv = nU + qp.nx[0]
    X = [np.hstack([np.zeros((qp.nx[0], nU)), np.eye(qp.nx[0])])]
    c = [np.zeros(qp.nx[0])]
    for n in range(N):
        S = np.zeros((qp.nu[n], nv))
        S[:, off[n]:off[n] + qp.nu[n]] = np.eye(qp.nu[n])
        A = np.asarray(qp.A[n]).reshape(qp.nx[n + 1], qp.nx[n])
        B = np.asarray(qp.B[n]).reshape(qp.nx[n + 1], qp.nu[n])
        X.append(A @ X[n] + B @ S)
        c.append(A @ c[n] + np.asarray(qp.b[n]))
    return X, c, off, nv


def condense_dense(qp):
    """The dense QP of full condensing: H, g, box rows (index into v, lower,
    upper) and general rows (C, lower, upper)."""
    N = qp.N
    X, c, off, nv = state_maps(qp)
    H = np.zeros((nv, nv))
    g = np.zeros(nv)
    bidx, blo, bhi = [], [], []
    rows, rlo, rhi = [], [], []
    for n in range(N + 1):
        nu, nx = qp.nu[n], qp.nx[n]
        S = np.zeros((nu, nv))
        if nu > 0:
            S[:, off[n]:off[n] + nu] = np.eye(nu)
        E = np.vstack([S, X[n]])
        e = np.concatenate([np.zeros(nu), c[n]])
        Hn = _stage_H(qp, n)
        gn = np.concatenate([np.asarray(qp.r[n]).ravel(), np.asarray(qp.q[n]).ravel()])
        H += E.T @ Hn @ E
        g += E.T @ (Hn @ e + gn)
        for j, i in enumerate(np.asarray(qp.idxbu[n], dtype=int)):
            bidx.append(off[n] + i)
            blo.append(qp.lbu[n][j])
            bhi.append(qp.ubu[n][j])
        for j, i in enumerate(np.asarray(qp.idxbx[n], dtype=int)):
            if n == 0:
                bidx.append(off[N + 1] + i)
                blo.append(qp.lbx[n][j])
                bhi.append(qp.ubx[n][j])
            else:
                rows.append(X[n][i, :])
                rlo.append(qp.lbx[n][j] - c[n][i])
                rhi.append(qp.ubx[n][j] - c[n][i])
        Dn = np.asarray(qp.D[n]).reshape(-1, nu) if nu > 0 else np.zeros((np.asarray(qp.D[n]).shape[0], 0))
        Cn = np.asarray(qp.C[n]).reshape(Dn.shape[0], nx)
        for j in range(Dn.shape[0]):
            rows.append(Dn[j] @ S + Cn[j] @ X[n])
            sh = Cn[j] @ c[n]
            rlo.append(qp.lg[n][j] - sh)
            rhi.append(qp.ug[n][j] - sh)
    return SimpleNamespace(nv=nv, H=0.5 * (H + H.T), g=g, bidx=np.asarray(bidx, dtype=int),
                           blo=np.asarray(blo, dtype=float), bhi=np.asarray(bhi, dtype=float),
                           C=np.asarray(rows, dtype=float).reshape(len(rows), nv), glo=np.asarray(rlo, dtype=float),
                           ghi=np.asarray(rhi, dtype=float), off=off)


def _rows(dq):
    """All rows of the dense QP as one matrix (boxes as unit rows first)."""
    Ab = np.zeros((len(dq.bidx), dq.nv))
    Ab[np.arange(len(dq.bidx)), dq.bidx] = 1.0
    return np.vstack([Ab, dq.C]), np.concatenate([dq.blo, dq.glo]), np.concatenate([dq.bhi, dq.ghi])


def residuals(dq, v, lam_l, lam_u, t_l, t_u):
    """r_g, r_d (lower, upper) of the dense QP and the four inf-norms."""
    A, lo, hi = _rows(dq)
    Av = A @ v
    rg = dq.H @ v + dq.g - A.T @ (lam_l - lam_u)
    rdl = t_l - (Av - lo)
    rdu = t_u - (hi - Av)
    rm = np.concatenate([lam_l * t_l, lam_u * t_u])
    norms = np.array([np.max(np.abs(rg), initial=0.0), 0.0,
                      max(np.max(np.abs(rdl), initial=0.0), np.max(np.abs(rdu), initial=0.0)),
                      np.max(rm, initial=0.0)])
    return rg, rdl, rdu, norms


def solve_dense(dq, tol: float = 1e-8, iter_max: int = 100, gamma: float = 0.995, alpha_min: float = 1e-10,
                corr_ratio: float = 10.0, clamp: float = 1e-16, sigma_pow: float = 3.0, corrector: bool = True):
    """The IPM on the dense QP.  Returns (status, iters, v, lam_l, lam_u,
    t_l, t_u, norms); status 0 success, 1 max iterations, 2 too short a step,
    3 NaN (the OCP oracle's codes).  sigma_pow and corrector exist only so
    that tests can show the trajectory comparison notices a change of the
    centering rule or a dropped corrector (sigma = (mu_aff / mu)^3 and the
    conditional corrector are the method)."""
    A, lo, hi = _rows(dq)
    m = A.shape[0]
    v = np.zeros(dq.nv)
    Av = A @ v
    t_l = np.maximum(Av - lo, 1.0)
    t_u = np.maximum(hi - Av, 1.0)
    lam_l = np.ones(m)
    lam_u = np.ones(m)
    nc2 = 2.0 * m
    for k in range(iter_max + 1):
        rg, rdl, rdu, norms = residuals(dq, v, lam_l, lam_u, t_l, t_u)
        mu = (lam_l @ t_l + lam_u @ t_u) / nc2 if m > 0 else 0.0
        if not np.all(np.isfinite(norms)):
            return 3, k, v, lam_l, lam_u, t_l, t_u, norms
        if norms[0] <= tol and norms[2] <= tol and norms[3] <= tol:
            return 0, k, v, lam_l, lam_u, t_l, t_u, norms
        if k == iter_max:
            return 1, k, v, lam_l, lam_u, t_l, t_u, norms
        w = lam_l / t_l + lam_u / t_u
        L = np.linalg.cholesky(dq.H + (A.T * w) @ A)

        def step(rml, rmu):
            # eliminate dt, dlam: dlam_l - dlam_u = -w A dv + e
            e = (lam_l * rdl - rml) / t_l - (lam_u * rdu - rmu) / t_u
            dv = -sla.cho_solve((L, True), rg - A.T @ e)
            Adv = A @ dv
            dtl = Adv - rdl
            dtu = -Adv - rdu
            dll = -(rml + lam_l * dtl) / t_l
            dlu = -(rmu + lam_u * dtu) / t_u
            return dv, dll, dlu, dtl, dtu

        def amax(dll, dlu, dtl, dtu):
            a = np.inf
            for x, dx in ((lam_l, dll), (lam_u, dlu), (t_l, dtl), (t_u, dtu)):
                neg = dx < 0
                if np.any(neg):
                    a = min(a, float(np.min(-x[neg] / dx[neg])))
            return a

        def mu_at(a, dll, dlu, dtl, dtu):
            return ((lam_l + a * dll) @ (t_l + a * dtl) + (lam_u + a * dlu) @ (t_u + a * dtu)) / nc2

        # predictor (affine step)
        aff = step(lam_l * t_l, lam_u * t_u)
        a_aff = min(1.0, amax(*aff[1:]))
        mu_aff = max(0.0, mu_at(a_aff, *aff[1:])) if m > 0 else 0.0
        sigma_mu = (mu_aff / mu) ** sigma_pow * mu if mu > 0 else 0.0
        # corrector, rejected for the predictor-centering step when it raises
        # the duality measure too much (Section 4.2)
        st = step(lam_l * t_l + aff[1] * aff[3] - sigma_mu, lam_u * t_u + aff[2] * aff[4] - sigma_mu)
        a_c = min(1.0, amax(*st[1:]))
        if not corrector or (m > 0 and mu_at(a_c, *st[1:]) > corr_ratio * mu_aff):
            st = step(lam_l * t_l - sigma_mu, lam_u * t_u - sigma_mu)
        a = min(1.0, gamma * amax(*st[1:]))
        dv, dll, dlu, dtl, dtu = st
        v = v + a * dv
        lam_l = np.maximum(lam_l + a * dll, clamp)
        lam_u = np.maximum(lam_u + a * dlu, clamp)
        t_l = np.maximum(t_l + a * dtl, clamp)
        t_u = np.maximum(t_u + a * dtu, clamp)
        if a < alpha_min:
            rg, rdl, rdu, norms = residuals(dq, v, lam_l, lam_u, t_l, t_u)
            return 2, k + 1, v, lam_l, lam_u, t_l, t_u, norms
    raise AssertionError("unreachable")


def expand_dense(qp, v) -> Dict[str, np.ndarray]:
    """Inputs and states of the original QP from the dense variables."""
    X, c, off, nv = state_maps(qp)
    u = np.concatenate([v[off[n]:off[n] + qp.nu[n]] for n in range(qp.N + 1)])
    x = np.concatenate([X[n] @ v + c[n] for n in range(qp.N + 1)])
    return {"u": u, "x": x}


def solve(qp, tol: float = 1e-8, iter_max: int = 100):
    """Full condensing, the dense IPM, expansion: (status, iters, {"u", "x"},
    norms of the dense QP)."""
    dq = condense_dense(qp)
    st, k, v, *_, norms = solve_dense(dq, tol=tol, iter_max=iter_max)
    return st, k, expand_dense(qp, v), norms
