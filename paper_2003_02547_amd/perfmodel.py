"""Algorithmic work model of one IPM iteration (what the method must move and
compute, independent of any implementation's extra traffic).

Bytes: the FP64 problem data of an instance, read once per residual
evaluation of eq:alg:pdipm:delta (one per iteration plus the final check,
plus one per refinement step in the mixed path).

Flops per iteration (multiply-add = 2 flops), per stage with
nz = nu + nx and nx' = nx of the next stage:
  factorization: nx'^2 nz + nz (nz+1) nx' + nz^3 / 3 + ng nu (nu + 1)
  two solves:    2 [4 nz nx' + 2 nz^2 + 4 ng nu]
  one residual:  2 nz^2 + 4 nx' nz + 4 ng nu
and per refinement correction (Section 3.4) one residual of the Newton
system and one solve with the stored factors:
  correction:    [4 nz nx' + 2 nz^2 + 4 ng nu] + [2 nz^2 + 4 nx' nz + 4 ng nu]
"""
from __future__ import annotations

import numpy as np


def data_bytes(qp) -> int:
    """FP64 problem data of one instance in its unpadded form (index lists
    counted as int32)."""
    n8 = 0
    n4 = 0
    for n in range(qp.N + 1):
        nx, nu = qp.nx[n], qp.nu[n]
        if n < qp.N:
            nxn = qp.nx[n + 1]
            n8 += nxn * nx + nxn * nu + nxn
        n8 += nx * nx + nu * nx + nu * nu + nx + nu
        nbu, nbx, ng = len(qp.idxbu[n]), len(qp.idxbx[n]), np.asarray(qp.D[n]).shape[0]
        n8 += 2 * (nbu + nbx) + ng * (nu + nx) + 2 * ng
        n4 += nbu + nbx
    return 8 * n8 + 4 * n4


def flops_per_iter(qp) -> float:
    f = 0.0
    for n in range(qp.N + 1):
        nx, nu = qp.nx[n], qp.nu[n]
        nz = nx + nu
        nxn = qp.nx[n + 1] if n < qp.N else 0
        ng = np.asarray(qp.D[n]).shape[0]
        fact = nxn * nxn * nz + nz * (nz + 1) * nxn + nz ** 3 / 3.0 + ng * nu * (nu + 1)
        solves = 2 * (4 * nz * nxn + 2 * nz * nz + 4 * ng * nu)
        resid = 2 * nz * nz + 4 * nxn * nz + 4 * ng * nu
        f += fact + solves + resid
    return f


def flops_per_refinement(qp) -> float:
    f = 0.0
    for n in range(qp.N + 1):
        nx, nu = qp.nx[n], qp.nu[n]
        nz = nx + nu
        nxn = qp.nx[n + 1] if n < qp.N else 0
        ng = np.asarray(qp.D[n]).shape[0]
        f += (4 * nz * nxn + 2 * nz * nz + 4 * ng * nu) + (2 * nz * nz + 4 * nxn * nz + 4 * ng * nu)
    return f
