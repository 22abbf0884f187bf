"""Partial condensing of an OCP QP and expansion of its solution (Section 3.5).

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU baseline
use it; the GPU path never does, and nothing here imports the GPU package.

Partial condensing turns an OCP QP with horizon N into one with horizon
N2 < N by grouping consecutive stages into blocks and eliminating every state
inside a block through the dynamics; only the state at the first stage of a
block stays a variable (Section 3.5).  What is computed follows from that
definition, written out with dense numpy algebra:

* blocks: stages [s_b, s_{b+1}) for b = 0..N2-1, with N = q N2 + r split into
  near-equal blocks, the first r of them one stage longer; stage N alone is
  the terminal stage of the condensed QP;
* condensed variables of block b: u_bar = [u_{s_b}; ...; u_{s_{b+1}-1}] and
  x_bar = x_{s_b};
* inside the block, the stacked states x_{s_b+1..s_{b+1}} are the solution of
  the block-bidiagonal system x_{k+1} - A_k x_k = B_k u_k + b_k with x_{s_b}
  = x_bar, solved here by one dense linear solve; that gives the affine maps
  x_k = Gam_k [u_bar; x_bar] + gam_k;
* condensed cost: sum over the block of the stage costs at those maps;
  condensed dynamics: x_{s_{b+1}} = Gam_{end} [u_bar; x_bar] + gam_{end};
* constraints: input boxes stay boxes (at their offset in u_bar), the state
  box of the first stage stays a box, state boxes of later stages become
  general rows (row Gam_k[i, :], bounds shifted by gam_k[i]), general rows
  become D S_k + C Gam_k with bounds shifted by C gam_k.  Row order within a
  condensed stage: for each stage of the block in order, its state-box rows
  (later stages only, increasing component) then its general rows.  Box
  index lists of the condensed QP are in increasing component order.

Expansion maps a solution of the condensed QP back: inputs and block-start
states are read off, interior states follow from the dynamics, multipliers
and slacks of every constraint are those of its condensed row, the dynamics
multiplier at a block end is the condensed one, and interior dynamics
multipliers come from the state rows of the stationarity residual r_g of
eq:alg:pdipm:delta set to zero, solved backwards through the block.
"""
from __future__ import annotations

from types import SimpleNamespace
from typing import Dict, List

import numpy as np


def block_starts(N: int, N2: int) -> List[int]:
    """First stage of each block plus N (N2 + 1 entries); N2 is clipped to N."""
    if N2 < 1:
        raise ValueError("condensed horizon must be >= 1")
    N2 = min(N2, N)
    q, r = divmod(N, N2)
    s = [0]
    for b in range(N2):
        s.append(s[-1] + q + (1 if b < r else 0))
    assert s[-1] == N
    return s


def _stage_H(qp, n):
    nu, nx = qp.nu[n], qp.nx[n]
    H = np.zeros((nu + nx, nu + nx))
    H[:nu, :nu] = qp.R[n]
    H[:nu, nu:] = qp.S[n]
    H[nu:, :nu] = np.asarray(qp.S[n]).T
    H[nu:, nu:] = qp.Q[n]
    return H


def _block_maps(qp, s0: int, s1: int):
    """Affine maps x_k = Gam[k] zb + gam[k] for k = 0..len (k = len only when
    s1 <= N - 1 + 1, i.e. the block has dynamics at its end) from one dense
    solve of the block's dynamics."""
    nus = [qp.nu[n] for n in range(s0, s1)]
    nU = sum(nus)
    nxs = qp.nx[s0]
    nzb = nU + nxs
    off = np.concatenate([[0], np.cumsum(nus)]).astype(int)
    L = s1 - s0
    Gam = [np.hstack([np.zeros((nxs, nU)), np.eye(nxs)])]
    gam = [np.zeros(nxs)]
    if s1 > s0 and s1 - 1 < qp.N:
        # unknowns: x_{s0+1}, ..., x_{s1}
        sizes = [qp.nx[s0 + k] for k in range(1, L + 1)]
        o = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
        nX = int(o[-1])
        T = np.eye(nX)
        Rm = np.zeros((nX, nzb))
        rv = np.zeros(nX)
        for k in range(L):
            n = s0 + k
            rows = slice(o[k], o[k + 1])
            # x_{k+1} - A_k x_k = B_k u_k + b_k
            Rm[rows, off[k]:off[k] + nus[k]] = qp.B[n]
            rv[rows] = qp.b[n]
            if k == 0:
                Rm[rows, nU:] += qp.A[n]
            else:
                T[rows, o[k - 1]:o[k]] = -np.asarray(qp.A[n])
        sol = np.linalg.solve(T, np.hstack([Rm, rv[:, None]]))
        for k in range(1, L + 1):
            rows = slice(o[k - 1], o[k])
            Gam.append(sol[rows, :nzb])
            gam.append(sol[rows, nzb])
    return Gam, gam, off, nU, nxs


def condense(qp, N2: int):
    """The partially condensed QP (same field names as the input)."""
    N = qp.N
    s = block_starts(N, N2)
    N2 = len(s) - 1
    out = {k: [] for k in ("nx", "nu", "A", "B", "b", "Q", "S", "R", "q", "r", "idxbu", "lbu", "ubu",
                           "idxbx", "lbx", "ubx", "D", "C", "lg", "ug")}
    blocks = [(s[b], s[b + 1]) for b in range(N2)] + [(N, N + 1)]
    for b, (s0, s1) in enumerate(blocks):
        Gam, gam, off, nU, nxs = _block_maps(qp, s0, s1)
        nzb = nU + nxs
        Hb = np.zeros((nzb, nzb))
        gb = np.zeros(nzb)
        iu, lu, hu = [], [], []
        rows, rlo, rhi = [], [], []
        for k in range(s1 - s0):
            n = s0 + k
            nu, nx = qp.nu[n], qp.nx[n]
            E = np.zeros((nu + nx, nzb))
            E[:nu, off[k]:off[k] + nu] = np.eye(nu)
            E[nu:, :] = Gam[k]
            e = np.concatenate([np.zeros(nu), gam[k]])
            H = _stage_H(qp, n)
            g = np.concatenate([qp.r[n], qp.q[n]])
            Hb += E.T @ H @ E
            gb += E.T @ (H @ e + g)
            p = np.argsort(qp.idxbu[n], kind="stable")
            iu += list(off[k] + np.asarray(qp.idxbu[n])[p])
            lu += list(np.asarray(qp.lbu[n])[p])
            hu += list(np.asarray(qp.ubu[n])[p])
            if k >= 1:
                p = np.argsort(qp.idxbx[n], kind="stable")
                for j in p:
                    i = int(qp.idxbx[n][j])
                    rows.append(Gam[k][i, :])
                    rlo.append(qp.lbx[n][j] - gam[k][i])
                    rhi.append(qp.ubx[n][j] - gam[k][i])
            Dn, Cn = np.asarray(qp.D[n]), np.asarray(qp.C[n])
            for j in range(Dn.shape[0]):
                row = np.zeros(nzb)
                row[off[k]:off[k] + nu] = Dn[j]
                row += Cn[j] @ Gam[k]
                rows.append(row)
                sh = Cn[j] @ gam[k]
                rlo.append(qp.lg[n][j] - sh)
                rhi.append(qp.ug[n][j] - sh)
        out["nx"].append(nxs)
        out["nu"].append(nU)
        out["R"].append(Hb[:nU, :nU])
        out["S"].append(Hb[:nU, nU:])
        out["Q"].append(Hb[nU:, nU:])
        out["r"].append(gb[:nU])
        out["q"].append(gb[nU:])
        if b < N2:
            F = Gam[-1]
            out["B"].append(F[:, :nU])
            out["A"].append(F[:, nU:])
            out["b"].append(gam[-1])
        out["idxbu"].append(np.asarray(iu, dtype=np.int32))
        out["lbu"].append(np.asarray(lu, dtype=np.float64))
        out["ubu"].append(np.asarray(hu, dtype=np.float64))
        p = np.argsort(qp.idxbx[s0], kind="stable")
        out["idxbx"].append(np.asarray(qp.idxbx[s0], dtype=np.int32)[p])
        out["lbx"].append(np.asarray(qp.lbx[s0], dtype=np.float64)[p])
        out["ubx"].append(np.asarray(qp.ubx[s0], dtype=np.float64)[p])
        G = np.asarray(rows, dtype=np.float64).reshape(len(rows), nzb)
        out["D"].append(G[:, :nU])
        out["C"].append(G[:, nU:])
        out["lg"].append(np.asarray(rlo, dtype=np.float64))
        out["ug"].append(np.asarray(rhi, dtype=np.float64))
    return SimpleNamespace(N=N2, meta={"blocks": s}, **out)


def _split(v, sizes):
    o = np.concatenate([[0], np.cumsum(sizes)]).astype(int)
    return [np.asarray(v[o[i]:o[i + 1]]) for i in range(len(sizes))]


def expand(qp, N2: int, csol: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    """Solution of the original QP from a solution of condense(qp, N2)."""
    N = qp.N
    cq = condense(qp, N2)
    s = block_starts(N, N2)
    N2 = len(s) - 1
    nbu = [len(i) for i in qp.idxbu]
    nbx = [len(i) for i in qp.idxbx]
    ng = [np.asarray(d).shape[0] for d in qp.D]
    cnbu = [len(i) for i in cq.idxbu]
    cnbx = [len(i) for i in cq.idxbx]
    cng = [d.shape[0] for d in cq.D]
    cu = _split(csol["u"], cq.nu)
    cx = _split(csol["x"], cq.nx)
    cpi = _split(csol["pi"], cq.nx[1:])
    cc = {k: _split(csol[k], [a + b + c for a, b, c in zip(cnbu, cnbx, cng)]) for k in ("lam_l", "lam_u", "t_l", "t_u")}
    u = [None] * (N + 1)
    x = [None] * (N + 1)
    pi = [None] * (N + 1)  # pi[n] multiplies the dynamics n-1 -> n
    con = {k: [None] * (N + 1) for k in cc}
    blocks = [(s[b], s[b + 1]) for b in range(N2)] + [(N, N + 1)]
    for b, (s0, s1) in enumerate(blocks):
        nus = [qp.nu[n] for n in range(s0, s1)]
        off = np.concatenate([[0], np.cumsum(nus)]).astype(int)
        for k in range(s1 - s0):
            n = s0 + k
            u[n] = cu[b][off[k]:off[k] + nus[k]]
            x[n] = cx[b] if k == 0 else qp.A[n - 1] @ x[n - 1] + qp.B[n - 1] @ u[n - 1] + qp.b[n - 1]
        # constraint vectors: condensed stage b = [box u | box x | general]
        gi = cnbu[b] + cnbx[b]  # next condensed general row
        for k in range(s1 - s0):
            n = s0 + k
            parts = {key: np.zeros(nbu[n] + nbx[n] + ng[n]) for key in cc}
            # input boxes: the condensed box list is sorted by component
            cidx = list(cq.idxbu[b])
            for j in range(nbu[n]):
                c = cidx.index(off[k] + int(qp.idxbu[n][j]))
                for key in cc:
                    parts[key][j] = cc[key][b][c]
            order = np.argsort(qp.idxbx[n], kind="stable")
            if k == 0:
                cxi = list(cq.idxbx[b])
                for j in range(nbx[n]):
                    c = cnbu[b] + cxi.index(int(qp.idxbx[n][j]))
                    for key in cc:
                        parts[key][nbu[n] + j] = cc[key][b][c]
            else:
                for pos, j in enumerate(order):
                    for key in cc:
                        parts[key][nbu[n] + j] = cc[key][b][gi + pos]
                gi += nbx[n]
            for j in range(ng[n]):
                for key in cc:
                    parts[key][nbu[n] + nbx[n] + j] = cc[key][b][gi + j]
            gi += ng[n]
            for key in cc:
                con[key][n] = parts[key]
    # interior dynamics multipliers: zero state rows of r_g, backwards per block
    for b in range(N2):
        s0, s1 = s[b], s[b + 1]
        pi[s1] = cpi[b]
        for n in range(s1 - 1, s0, -1):
            nu = qp.nu[n]
            H = _stage_H(qp, n)
            z = np.concatenate([u[n], x[n]])
            v = (H @ z)[nu:] + qp.q[n] + np.asarray(qp.A[n]).T @ pi[n + 1]
            dl = con["lam_l"][n] - con["lam_u"][n]
            for j in range(nbx[n]):
                v[int(qp.idxbx[n][j])] -= dl[nbu[n] + j]
            if ng[n]:
                v -= np.asarray(qp.C[n]).T @ dl[nbu[n] + nbx[n]:]
            pi[n] = v
    cat = lambda L: np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in L]) if L else np.zeros(0)
    return {
        "u": cat(u), "x": cat(x), "pi": cat(pi[1:]),
        **{key: cat(con[key]) for key in con},
    }
