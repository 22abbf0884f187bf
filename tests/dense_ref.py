"""Dense, definition-level references used to pin the oracle.

Everything here is built directly from the problem statement with numpy /
scipy routines, independently of the oracle's stage-wise recursion:

  * the generic-QP matrices of eq:alg:pdipm:qp for an OCP QP (Section 2.2),
    with the two-sided rows stacked as C = [G; -G], d = [lo; -hi];
  * the residual function and the full 4-block Newton matrix of
    eq:alg:pdipm:delta, solved by dense LU (numpy.linalg.solve);
  * brute-force enumeration of active sets for tiny QPs (the unique
    minimiser of a strictly convex QP, the result the IPM approaches);
  * the textbook finite-horizon LQR recursion and the discrete algebraic
    Riccati equation (scipy.linalg.solve_discrete_are).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg


class DenseQp:
    """min 1/2 y'Hy + g'y  s.t.  Aeq y = beq,  lo <= G y <= hi, with y the
    stage-wise concatenation of [u_n; x_n] and constraint rows per stage in
    the order [box u, box x, general]."""

    def __init__(self, qp):
        N = qp.N
        nz = [qp.nx[n] + qp.nu[n] for n in range(N + 1)]
        zoff = np.concatenate([[0], np.cumsum(nz)]).astype(int)
        nv = int(zoff[-1])
        H = np.zeros((nv, nv)); g = np.zeros(nv)
        neq = sum(qp.nx[n + 1] for n in range(N))
        Aeq = np.zeros((neq, nv)); beq = np.zeros(neq)
        rows, lo, hi = [], [], []
        e = 0
        for n in range(N + 1):
            nu, nx = qp.nu[n], qp.nx[n]
            z0 = zoff[n]
            Hn = np.zeros((nu + nx, nu + nx))
            Hn[:nu, :nu] = qp.R[n]
            Hn[:nu, nu:] = qp.S[n]
            Hn[nu:, :nu] = np.asarray(qp.S[n]).T
            Hn[nu:, nu:] = qp.Q[n]
            H[z0:z0 + nu + nx, z0:z0 + nu + nx] = Hn
            g[z0:z0 + nu] = qp.r[n]
            g[z0 + nu:z0 + nu + nx] = qp.q[n]
            if n < N:
                nxn = qp.nx[n + 1]
                # x_{n+1} - A x_n - B u_n = b_n
                Aeq[e:e + nxn, z0:z0 + nu] = -np.asarray(qp.B[n])
                Aeq[e:e + nxn, z0 + nu:z0 + nu + nx] = -np.asarray(qp.A[n])
                z1 = zoff[n + 1] + qp.nu[n + 1]
                Aeq[e:e + nxn, z1:z1 + nxn] = np.eye(nxn)
                beq[e:e + nxn] = qp.b[n]
                e += nxn
            for k, j in enumerate(qp.idxbu[n]):
                row = np.zeros(nv); row[z0 + j] = 1.0
                rows.append(row); lo.append(qp.lbu[n][k]); hi.append(qp.ubu[n][k])
            for k, j in enumerate(qp.idxbx[n]):
                row = np.zeros(nv); row[z0 + nu + j] = 1.0
                rows.append(row); lo.append(qp.lbx[n][k]); hi.append(qp.ubx[n][k])
            Dn, Cn = np.asarray(qp.D[n]), np.asarray(qp.C[n])
            for k in range(Dn.shape[0]):
                row = np.zeros(nv)
                row[z0:z0 + nu] = Dn[k]
                row[z0 + nu:z0 + nu + nx] = Cn[k]
                rows.append(row); lo.append(qp.lg[n][k]); hi.append(qp.ug[n][k])
        self.qp = qp
        self.N = N
        self.zoff = zoff
        self.nv, self.neq = nv, neq
        self.H, self.g, self.Aeq, self.beq = H, g, Aeq, beq
        self.G = np.array(rows).reshape(len(rows), nv)
        self.lo, self.hi = np.array(lo), np.array(hi)
        self.m = len(rows)
        # generic-QP inequality C y >= d
        self.Cin = np.vstack([self.G, -self.G])
        self.d = np.concatenate([self.lo, -self.hi])

    # user layout <-> stacked vectors -------------------------------------
    def y_from(self, u, x):
        y = np.zeros(self.nv)
        ou = ox = 0
        for n in range(self.N + 1):
            nu, nx = self.qp.nu[n], self.qp.nx[n]
            y[self.zoff[n]:self.zoff[n] + nu] = u[ou:ou + nu]
            y[self.zoff[n] + nu:self.zoff[n] + nu + nx] = x[ox:ox + nx]
            ou += nu; ox += nx
        return y

    def ux_from(self, y):
        u, x = [], []
        for n in range(self.N + 1):
            nu, nx = self.qp.nu[n], self.qp.nx[n]
            u.append(y[self.zoff[n]:self.zoff[n] + nu])
            x.append(y[self.zoff[n] + nu:self.zoff[n] + nu + nx])
        return np.concatenate(u) if u else np.zeros(0), np.concatenate(x) if x else np.zeros(0)

    def stack(self, it):
        y = self.y_from(it["u"], it["x"])
        lam = np.concatenate([it["lam_l"], it["lam_u"]])
        t = np.concatenate([it["t_l"], it["t_u"]])
        return y, np.asarray(it["pi"], dtype=float), lam, t

    # eq:alg:pdipm:delta ----------------------------------------------------
    def residual(self, it, tau=0.0):
        y, pi, lam, t = self.stack(it)
        rg = self.H @ y + self.g - self.Aeq.T @ pi - self.Cin.T @ lam
        rb = -self.Aeq @ y + self.beq
        rd = -self.Cin @ y + t + self.d
        rm = lam * t - tau
        return rg, rb, rd, rm

    def kkt_matrix(self, it):
        _, _, lam, t = self.stack(it)
        nv, ne, nc = self.nv, self.neq, 2 * self.m
        K = np.zeros((nv + ne + 2 * nc, nv + ne + 2 * nc))
        a, b, c = nv, nv + ne, nv + ne + nc
        K[:a, :a] = self.H
        K[:a, a:b] = -self.Aeq.T
        K[:a, b:c] = -self.Cin.T
        K[a:b, :a] = -self.Aeq
        K[b:c, :a] = -self.Cin
        K[b:c, c:] = np.eye(nc)
        K[c:, b:c] = np.diag(t)
        K[c:, c:] = np.diag(lam)
        return K

    def newton_step(self, it, tau=0.0):
        rg, rb, rd, rm = self.residual(it, tau)
        K = self.kkt_matrix(it)
        sol = np.linalg.solve(K, -np.concatenate([rg, rb, rd, rm]))
        return self.unstack_step(sol)

    def unstack_step(self, sol):
        nv, ne, m = self.nv, self.neq, self.m
        dy = sol[:nv]; dpi = sol[nv:nv + ne]
        dlam = sol[nv + ne:nv + ne + 2 * m]; dt = sol[nv + ne + 2 * m:]
        du, dx = self.ux_from(dy)
        return dict(u=du, x=dx, pi=dpi, lam_l=dlam[:m], lam_u=dlam[m:], t_l=dt[:m], t_u=dt[m:])

    def reduced_step(self, it, tau=0.0):
        """The same step through the reduced system eq:alg:kkt (dense)."""
        y, pi, lam, t = self.stack(it)
        rg, rb, rd, rm = self.residual(it, tau)
        W = lam / t
        Phi = self.H + self.Cin.T @ np.diag(W) @ self.Cin
        gt = rg - self.Cin.T @ (W * rd - rm / t)
        nv, ne = self.nv, self.neq
        Kr = np.zeros((nv + ne, nv + ne))
        Kr[:nv, :nv] = Phi; Kr[:nv, nv:] = -self.Aeq.T; Kr[nv:, :nv] = -self.Aeq
        s = np.linalg.solve(Kr, -np.concatenate([gt, rb]))
        dy, dpi = s[:nv], s[nv:]
        dt = self.Cin @ dy - rd
        dlam = -(rm + lam * dt) / t
        m = self.m
        du, dx = self.ux_from(dy)
        return dict(u=du, x=dx, pi=dpi, lam_l=dlam[:m], lam_u=dlam[m:], t_l=dt[:m], t_u=dt[m:])

    # exact minimiser by brute force -----------------------------------------
    def brute_force(self, tol=1e-9):
        """Enumerate {inactive, lower, upper} per two-sided row (equal-limit
        rows are always active, with a free-sign multiplier); keep the
        primal-feasible, dual-feasible equality-QP solutions.  Returns the
        list of certified y (all equal for a strictly convex QP)."""
        m = self.m
        fixed = np.isclose(self.lo, self.hi, rtol=0, atol=0)
        free_rows = [i for i in range(m) if not fixed[i]]
        found = []
        for states in itertools.product((0, -1, 1), repeat=len(free_rows)):
            act, val, sign = [], [], []
            for i in range(m):
                if fixed[i]:
                    act.append(i); val.append(self.lo[i]); sign.append(0)
            for i, s in zip(free_rows, states):
                if s == -1:
                    act.append(i); val.append(self.lo[i]); sign.append(1)
                elif s == 1:
                    act.append(i); val.append(self.hi[i]); sign.append(-1)
            Ae = np.vstack([self.Aeq, self.G[act]]) if act else self.Aeq
            be = np.concatenate([self.beq, val]) if act else self.beq
            ne = Ae.shape[0]
            if ne > self.nv:
                continue
            K = np.zeros((self.nv + ne, self.nv + ne))
            K[:self.nv, :self.nv] = self.H
            K[:self.nv, self.nv:] = -Ae.T
            K[self.nv:, :self.nv] = Ae
            if np.linalg.matrix_rank(Ae) < ne:
                continue
            s = np.linalg.solve(K, np.concatenate([-self.g, be]))
            y, nu_ = s[:self.nv], s[self.nv:]
            Gy = self.G @ y
            if np.any(Gy < self.lo - tol) or np.any(Gy > self.hi + tol):
                continue
            mult = nu_[self.neq:]
            ok = True
            for mm, sg in zip(mult, sign):
                if sg == 1 and mm < -tol:
                    ok = False
                if sg == -1 and mm > tol:
                    ok = False
            if ok:
                found.append(y)
        return found


def lqr_finite_horizon(A, B, Q, R, QN, N, x0):
    """Textbook LQR: P_N = QN, K_n = (R + B'P B)^{-1} B'P A,
    P_n = Q + A'P (A - B K_n); u_n = -K_n x_n.  Returns (u list, x list)."""
    P = QN.copy()
    Ks = [None] * N
    for n in range(N - 1, -1, -1):
        K = np.linalg.solve(R + B.T @ P @ B, B.T @ P @ A)
        Ks[n] = K
        P = Q + A.T @ P @ (A - B @ K)
    xs, us = [x0.copy()], []
    for n in range(N):
        u = -Ks[n] @ xs[-1]
        us.append(u)
        xs.append(A @ xs[-1] + B @ u)
    return us, xs, Ks


def dare_gain(A, B, Q, R):
    P = scipy.linalg.solve_discrete_are(A, B, Q, R)
    K = np.linalg.solve(R + B.T @ P @ B, B.T @ P @ A)
    return P, K


def random_interior_iterate(qp, rng, scale=1.0):
    """A random point with lam, t > 0 (not necessarily feasible)."""
    nu, nx = sum(qp.nu), sum(qp.nx)
    npi = sum(qp.nx[1:])
    nc = qp.n_constraints()
    return dict(u=rng.standard_normal(nu) * scale, x=rng.standard_normal(nx) * scale,
                pi=rng.standard_normal(npi) * scale,
                lam_l=rng.uniform(0.1, 2.0, nc), lam_u=rng.uniform(0.1, 2.0, nc),
                t_l=rng.uniform(0.1, 2.0, nc), t_u=rng.uniform(0.1, 2.0, nc))


class DenseSoftQp:
    """The OCP QP with soft constraints (Section 2.2) as a generic QP in the
    augmented variables y' = [y; s^l; s^u], built from the definition with
    numpy, without eliminating the slacks:

      min 1/2 y'H y + g'y + sum_j 1/2 Zl_j (s^l_j)^2 + zl_j s^l_j + (same for s^u)
      s.t. Aeq y = beq,
           G_i y + s^l_j >= lo_i,  -G_i y + s^u_j >= -hi_i   (row i softened by slack j)
           G_i y >= lo_i,          -G_i y >= -hi_i            (hard rows)
           s^l >= lls,  s^u >= lus.

    One-sided rows are stacked [lower rows; upper rows; s^l bounds; s^u
    bounds], matching the user layout (lam_l, lam_u, lam_sl, lam_su) and
    (t_l, t_u, t_sl, t_su)."""

    def __init__(self, qp):
        base = DenseQp(qp)
        self.base = base
        self.qp = qp
        m, nv = base.m, base.nv
        coff = np.concatenate([[0], np.cumsum([qp.nbu[n] + qp.nbx[n] + qp.ng[n] for n in range(qp.N + 1)])])
        rows = []   # global constraint row of each slack, stage by stage in idxs order
        Zl, Zu, zl, zu, lls, lus = ([] for _ in range(6))
        for n in range(qp.N + 1):
            for j, k in enumerate(qp.idxs[n]):
                rows.append(int(coff[n] + k))
                Zl.append(qp.Zl[n][j]); Zu.append(qp.Zu[n][j]); zl.append(qp.zl[n][j]); zu.append(qp.zu[n][j])
                lls.append(qp.lls[n][j]); lus.append(qp.lus[n][j])
        ns = len(rows)
        self.m, self.ns, self.nv0 = m, ns, nv
        self.nv = nv + 2 * ns
        self.neq = base.neq
        self.H = scipy.linalg.block_diag(base.H, np.diag(Zl), np.diag(Zu)) if ns else base.H.copy()
        self.g = np.concatenate([base.g, zl, zu])
        self.Aeq = np.hstack([base.Aeq, np.zeros((base.neq, 2 * ns))])
        self.beq = base.beq
        C = np.zeros((2 * m + 2 * ns, self.nv))
        C[:m, :nv] = base.G
        C[m:2 * m, :nv] = -base.G
        for j, i in enumerate(rows):
            C[i, nv + j] = 1.0
            C[m + i, nv + ns + j] = 1.0
            C[2 * m + j, nv + j] = 1.0
            C[2 * m + ns + j, nv + ns + j] = 1.0
        self.Cin = C
        self.d = np.concatenate([base.lo, -base.hi, lls, lus])
        self.soft_rows = rows
        self.lo, self.hi = base.lo, base.hi

    def stack(self, it):
        y = np.concatenate([self.base.y_from(it["u"], it["x"]), it["s_l"], it["s_u"]])
        lam = np.concatenate([it["lam_l"], it["lam_u"], it["lam_sl"], it["lam_su"]])
        t = np.concatenate([it["t_l"], it["t_u"], it["t_sl"], it["t_su"]])
        return y, np.asarray(it["pi"], dtype=float), lam, t

    def residual(self, it, tau=0.0):
        y, pi, lam, t = self.stack(it)
        rg = self.H @ y + self.g - self.Aeq.T @ pi - self.Cin.T @ lam
        rb = -self.Aeq @ y + self.beq
        rd = -self.Cin @ y + t + self.d
        rm = lam * t - tau
        return rg, rb, rd, rm

    def split(self, vy, vc):
        """User-layout dict of a primal-sized and a row-sized vector pair."""
        m, ns, nv = self.m, self.ns, self.nv0
        u, x = self.base.ux_from(vy[:nv])
        return dict(u=u, x=x, s_l=vy[nv:nv + ns], s_u=vy[nv + ns:],
                    lam_l=vc[:m], lam_u=vc[m:2 * m], lam_sl=vc[2 * m:2 * m + ns], lam_su=vc[2 * m + ns:])

    def newton_step(self, it, tau=0.0):
        _, _, lam, t = self.stack(it)
        rg, rb, rd, rm = self.residual(it, tau)
        nv, ne, nc = self.nv, self.neq, self.Cin.shape[0]
        K = np.zeros((nv + ne + 2 * nc, nv + ne + 2 * nc))
        a, b, c = nv, nv + ne, nv + ne + nc
        K[:a, :a] = self.H
        K[:a, a:b] = -self.Aeq.T
        K[:a, b:c] = -self.Cin.T
        K[a:b, :a] = -self.Aeq
        K[b:c, :a] = -self.Cin
        K[b:c, c:] = np.eye(nc)
        K[c:, b:c] = np.diag(t)
        K[c:, c:] = np.diag(lam)
        sol = np.linalg.solve(K, -np.concatenate([rg, rb, rd, rm]))
        dy, dpi, dlam, dt = sol[:a], sol[a:b], sol[b:c], sol[c:]
        out = self.split(dy, dlam)
        tt = self.split(np.zeros(nv), dt)
        out.update(pi=dpi, t_l=tt["lam_l"], t_u=tt["lam_u"], t_sl=tt["lam_sl"], t_su=tt["lam_su"])
        return out

    def brute_force(self, tol=1e-9):
        """Enumerate active sets of the one-sided rows (hard rows with equal
        limits are equalities with a free-sign multiplier); keep the
        primal-feasible, dual-feasible equality-QP solutions.  Returns the
        certified y' (unique for Zl, Zu > 0)."""
        m, ns = self.m, self.ns
        soft = set(self.soft_rows)
        fixed = [i for i in range(m) if i not in soft and self.lo[i] == self.hi[i]]
        skip = set(fixed) | {m + i for i in fixed}
        free = [r for r in range(2 * m + 2 * ns) if r not in skip]
        found = []
        for states in itertools.product((0, 1), repeat=len(free)):
            act = [r for r, s in zip(free, states) if s]
            E = [self.Cin[i] for i in fixed] + [self.Cin[r] for r in act]
            ev = [self.lo[i] for i in fixed] + [self.d[r] for r in act]
            Ae = np.vstack([self.Aeq] + ([np.array(E)] if E else []))
            be = np.concatenate([self.beq, ev])
            ne = Ae.shape[0]
            if ne > self.nv or np.linalg.matrix_rank(Ae) < ne:
                continue
            K = np.zeros((self.nv + ne, self.nv + ne))
            K[:self.nv, :self.nv] = self.H
            K[:self.nv, self.nv:] = -Ae.T
            K[self.nv:, :self.nv] = Ae
            s = np.linalg.solve(K, np.concatenate([-self.g, be]))
            y, mult = s[:self.nv], s[self.nv + self.neq + len(fixed):]
            if np.any(self.Cin @ y < self.d - tol):
                continue
            if np.any(mult < -tol):
                continue
            found.append(y)
        return found


def random_interior_iterate_soft(qp, rng, scale=1.0):
    """random_interior_iterate plus slacks and positive slack-bound pairs."""
    it = random_interior_iterate(qp, rng, scale)
    ns = sum(len(i) for i in qp.idxs)
    it.update(s_l=rng.standard_normal(ns) * scale, s_u=rng.standard_normal(ns) * scale,
              lam_sl=rng.uniform(0.1, 2.0, ns), lam_su=rng.uniform(0.1, 2.0, ns),
              t_sl=rng.uniform(0.1, 2.0, ns), t_su=rng.uniform(0.1, 2.0, ns))
    return it
