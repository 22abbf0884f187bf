"""Python access to the plain FP64 CPU oracle (oqp_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline of the benchmark use it; the GPU path never does.  Nothing here
imports the GPU package: problems are passed in as any object with the
OcpQp fields (N, nx, nu, A, B, b, Q, S, R, q, r, idxbu, lbu, ubu, idxbx,
lbx, ubx, D, C, lg, ug).

The oracle implements the IPM of Section 4.2 (delta formulation, Mehrotra
predictor-corrector, conditional corrector, clamps) on the generic QP of
eq:alg:pdipm:qp with Newton steps of eq:alg:pdipm:delta solved through the
reduced system eq:alg:kkt and the classical Riccati recursion (Section 3.3).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oqp_oracle.c")
_LIB = os.path.join(_HERE, "liboqp_oracle.so")

SUCCESS, MAX_ITER, MIN_STEP, NAN = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (no BLAS, no intrinsics, no threads)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_P = ct.POINTER(ct.c_double)
_PI = ct.POINTER(ct.c_int)


class _Qp(ct.Structure):
    _fields_ = [("N", ct.c_int)] + [(n, _PI) for n in ("nx", "nu", "nbu", "nbx", "ng")] + \
        [(n, _P) for n in ("A", "B", "b", "Q", "S", "R", "q", "r")] + \
        [(n, _PI) for n in ("idxbu", "idxbx")] + \
        [(n, _P) for n in ("lbu", "ubu", "lbx", "ubx", "D", "C", "lg", "ug")] + \
        [("ns", _PI), ("idxs", _PI)] + [(n, _P) for n in ("Zl", "Zu", "zl", "zu", "lls", "lus")]


class _Arg(ct.Structure):
    _fields_ = [("tol_stat", ct.c_double), ("tol_eq", ct.c_double), ("tol_ineq", ct.c_double),
                ("tol_comp", ct.c_double), ("iter_max", ct.c_int), ("alpha_min", ct.c_double),
                ("gamma", ct.c_double), ("lam_min", ct.c_double), ("t_min", ct.c_double),
                ("reg_prim", ct.c_double), ("corr_ratio", ct.c_double), ("warm_start", ct.c_int),
                ("abs_form", ct.c_int), ("ir_max", ct.c_int), ("ir_tol", ct.c_double)]


SOFT_NAMES = ("s_l", "s_u", "lam_sl", "lam_su", "t_sl", "t_su")


class _Vec(ct.Structure):
    _fields_ = [(n, _P) for n in ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u") + SOFT_NAMES]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ct.CDLL(_LIB)
        lib.orc_solve.argtypes = [ct.POINTER(_Qp), ct.POINTER(_Arg), ct.POINTER(_Vec), _PI, _P, _P, _PI]
        lib.orc_solve.restype = ct.c_int
        lib.orc_residuals.argtypes = [ct.POINTER(_Qp), ct.POINTER(_Vec), ct.POINTER(_Vec), _P, _P]
        lib.orc_residuals.restype = ct.c_int
        lib.orc_newton_step.argtypes = [ct.POINTER(_Qp), ct.POINTER(_Vec), ct.c_double, ct.c_double, ct.c_int,
                                        ct.POINTER(_Vec)]
        lib.orc_newton_step.restype = ct.c_int
        lib.orc_newton_step_ir.argtypes = [ct.POINTER(_Qp), ct.POINTER(_Vec), ct.c_double, ct.c_double, ct.c_int,
                                           ct.c_double, ct.POINTER(_Vec), _PI]
        lib.orc_newton_step_ir.restype = ct.c_int
        lib.orc_ir_residual.argtypes = [ct.POINTER(_Qp), ct.POINTER(_Vec), ct.POINTER(_Vec),
                                        ct.POINTER(_Vec), ct.POINTER(_Vec)]
        lib.orc_ir_residual.restype = ct.c_int
        _lib = lib
    return _lib


@dataclass
class Arg:
    """IPM arguments (Section 4.2).  Defaults: the FP64 path."""
    tol_stat: float = 1e-8
    tol_eq: float = 1e-8
    tol_ineq: float = 1e-8
    tol_comp: float = 1e-8
    iter_max: int = 100
    alpha_min: float = 1e-10
    gamma: float = 0.995
    lam_min: float = 1e-16
    t_min: float = 1e-16
    reg_prim: float = 0.0
    corr_ratio: float = 10.0
    warm_start: int = 0  # 0 cold; 1 primal guess; 2 primal and dual guess (Section 4.2)
    abs_form: int = 0    # 1: absolute formulation (eq:alg:pdipm:abs), exit on the duality measure
    # refinement of the prediction-centering-correction direction (Sections
    # 3.4 and 4.2): up to ir_max corrections per direction, until the
    # refinement residual is within ir_tol * max(1, residual norms); 0: none
    ir_max: int = 0
    ir_tol: float = 1e-10

    def _c(self):
        return _Arg(self.tol_stat, self.tol_eq, self.tol_ineq, self.tol_comp, int(self.iter_max),
                    self.alpha_min, self.gamma, self.lam_min, self.t_min, self.reg_prim, self.corr_ratio,
                    int(self.warm_start), int(self.abs_form), int(self.ir_max), float(self.ir_tol))

    @staticmethod
    def with_tol(tol: float, **kw) -> "Arg":
        return Arg(tol_stat=tol, tol_eq=tol, tol_ineq=tol, tol_comp=tol, **kw)


def _cat(arrs, dtype=np.float64, order="F"):
    parts = [np.asarray(a, dtype=dtype).ravel(order=order) for a in arrs]
    if not parts:
        return np.zeros(1, dtype=dtype)
    out = np.concatenate(parts) if parts else np.zeros(0, dtype=dtype)
    return out if out.size else np.zeros(1, dtype=dtype)


class _Packed:
    """Flat concatenations of a problem, kept alive while the C call runs."""

    def __init__(self, qp):
        N = qp.N
        self.N = N
        self.nx = np.asarray(qp.nx, dtype=np.int32)
        self.nu = np.asarray(qp.nu, dtype=np.int32)
        self.nbu = np.asarray([len(i) for i in qp.idxbu], dtype=np.int32)
        self.nbx = np.asarray([len(i) for i in qp.idxbx], dtype=np.int32)
        self.ng = np.asarray([np.asarray(d).shape[0] for d in qp.D], dtype=np.int32)
        self.arrs = {
            "A": _cat(qp.A), "B": _cat(qp.B), "b": _cat(qp.b), "Q": _cat(qp.Q), "S": _cat(qp.S),
            "R": _cat(qp.R), "q": _cat(qp.q), "r": _cat(qp.r),
            "lbu": _cat(qp.lbu), "ubu": _cat(qp.ubu), "lbx": _cat(qp.lbx), "ubx": _cat(qp.ubx),
            "D": _cat(qp.D), "C": _cat(qp.C), "lg": _cat(qp.lg), "ug": _cat(qp.ug),
        }
        self.idxbu = _cat(qp.idxbu, np.int32)
        self.idxbx = _cat(qp.idxbx, np.int32)
        c = _Qp()
        c.N = N
        for k in ("nx", "nu", "nbu", "nbx", "ng"):
            setattr(c, k, getattr(self, k).ctypes.data_as(_PI))
        for k, v in self.arrs.items():
            setattr(c, k, v.ctypes.data_as(_P))
        c.idxbu = self.idxbu.ctypes.data_as(_PI)
        c.idxbx = self.idxbx.ctypes.data_as(_PI)
        # soft constraints (Section 2.2): absent unless the problem has idxs
        self.n_s = 0
        if getattr(qp, "idxs", None) is not None:
            self.ns = np.asarray([len(i) for i in qp.idxs], dtype=np.int32)
            self.idxs = _cat(qp.idxs, np.int32)
            self.soft = {k: _cat(getattr(qp, k)) for k in ("Zl", "Zu", "zl", "zu", "lls", "lus")}
            c.ns = self.ns.ctypes.data_as(_PI)
            c.idxs = self.idxs.ctypes.data_as(_PI)
            for k, v in self.soft.items():
                setattr(c, k, v.ctypes.data_as(_P))
            self.n_s = int(self.ns.sum())
        self.c = c
        self.n_u = int(self.nu.sum())
        self.n_x = int(self.nx.sum())
        self.n_pi = int(self.nx[1:].sum())
        self.n_c = int((self.nbu + self.nbx + self.ng).sum())


class Vec:
    """Iterate / step / residual in the user layout: u, x, pi and the per-stage
    constraint vectors ordered [box u, box x, general]; with soft constraints
    also the slacks s_l, s_u and the multipliers and slacks of their lower
    bounds (lam_sl, lam_su, t_sl, t_su), stage by stage in idxs order."""
    names = ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u") + SOFT_NAMES

    def __init__(self, n_u, n_x, n_pi, n_c, n_s=0):
        self.u = np.zeros(max(n_u, 1)); self.x = np.zeros(max(n_x, 1)); self.pi = np.zeros(max(n_pi, 1))
        self.lam_l = np.zeros(max(n_c, 1)); self.lam_u = np.zeros(max(n_c, 1))
        self.t_l = np.zeros(max(n_c, 1)); self.t_u = np.zeros(max(n_c, 1))
        for k in SOFT_NAMES:
            setattr(self, k, np.zeros(max(n_s, 1)))
        self._sizes = dict(u=n_u, x=n_x, pi=n_pi, lam_l=n_c, lam_u=n_c, t_l=n_c, t_u=n_c)
        self._sizes.update({k: n_s for k in SOFT_NAMES})
        self.n_s = n_s

    @classmethod
    def like(cls, pk: _Packed):
        return cls(pk.n_u, pk.n_x, pk.n_pi, pk.n_c, pk.n_s)

    def c(self):
        v = _Vec()
        for n in self.names:
            setattr(v, n, getattr(self, n).ctypes.data_as(_P))
        return v

    def view(self):
        """dict of arrays trimmed to their true sizes (the slack blocks only
        when the problem has slacks)."""
        names = self.names if self.n_s else self.names[:7]
        return {n: getattr(self, n)[: self._sizes[n]].copy() for n in names}

    def set(self, **kw):
        for k, v in kw.items():
            getattr(self, k)[: self._sizes[k]] = v
        return self


@dataclass
class Result:
    status: int
    iters: int
    res: np.ndarray   # inf-norms: stat, eq, ineq, comp
    mu: float
    sol: dict         # u, x, pi, lam_l, lam_u, t_l, t_u (and the slack blocks)
    ir_steps: int = 0  # refinement corrections kept in total


def solve(qp, arg: Arg | None = None, guess: dict | None = None) -> Result:
    """Run the oracle IPM on one problem; with arg.warm_start != 0 it starts
    from `guess` (user layout: u, x and, for warm_start = 2, pi, lam, t)."""
    lib = _load()
    arg = arg or Arg()
    pk = _Packed(qp)
    sol = Vec.like(pk)
    if guess is not None:
        sol.set(**{k: guess[k] for k in Vec.names if k in guess})
    it = ct.c_int(0)
    irs = ct.c_int(0)
    res = np.zeros(4)
    mu = ct.c_double(0.0)
    a = arg._c()
    sv = sol.c()
    st = lib.orc_solve(ct.byref(pk.c), ct.byref(a), ct.byref(sv), ct.byref(it),
                       res.ctypes.data_as(_P), ct.byref(mu), ct.byref(irs))
    if st < 0:
        raise ValueError(f"oracle rejected the problem (code {st})")
    return Result(st, it.value, res, mu.value, sol.view(), irs.value)


def _vec_from(pk, d):
    v = Vec.like(pk)
    v.set(**{k: d[k] for k in Vec.names if k in d})
    return v


def residuals(qp, iterate: dict):
    """Residuals (eq:alg:pdipm:delta RHS) at `iterate`.  Returns (parts, norms, mu):
    parts has r_g split into 'u'/'x' slots, r_b in 'pi', r_d lower/upper in
    'lam_l'/'lam_u', lam.*t lower/upper in 't_l'/'t_u'; with slacks, r_s in
    's_l'/'s_u', the slack bounds' r_d in 'lam_sl'/'lam_su' and their lam.*t
    in 't_sl'/'t_su'."""
    lib = _load()
    pk = _Packed(qp)
    it = _vec_from(pk, iterate)
    out = Vec.like(pk)
    norms = np.zeros(4)
    mu = ct.c_double(0.0)
    itc, outc = it.c(), out.c()
    rc = lib.orc_residuals(ct.byref(pk.c), ct.byref(itc), ct.byref(outc), norms.ctypes.data_as(_P), ct.byref(mu))
    if rc < 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    return out.view(), norms, mu.value


def newton_step(qp, iterate: dict, tau: float = 0.0, reg: float = 0.0, abs_form: bool = False) -> dict:
    """Newton step of eq:alg:pdipm:delta at `iterate`, r_m = lam.*t - tau; with
    abs_form the same step through the absolute formulation (eq:alg:pdipm:abs
    and eq:alg:pdipm:step)."""
    lib = _load()
    pk = _Packed(qp)
    it = _vec_from(pk, iterate)
    out = Vec.like(pk)
    itc, outc = it.c(), out.c()
    rc = lib.orc_newton_step(ct.byref(pk.c), ct.byref(itc), ct.c_double(tau), ct.c_double(reg), int(abs_form),
                             ct.byref(outc))
    if rc != 0:
        raise ValueError(f"oracle Newton step failed (code {rc})")
    return out.view()


def newton_step_refined(qp, iterate: dict, tau: float = 0.0, reg: float = 0.0, ir_max: int = 4,
                        ir_tol: float = 1e-10):
    """Newton step of eq:alg:pdipm:delta with iterative refinement (Section
    3.4): factorization with regularization reg, up to ir_max corrections
    against the unregularized matrix.  Returns (step, corrections kept)."""
    lib = _load()
    pk = _Packed(qp)
    it = _vec_from(pk, iterate)
    out = Vec.like(pk)
    kept = ct.c_int(0)
    itc, outc = it.c(), out.c()
    rc = lib.orc_newton_step_ir(ct.byref(pk.c), ct.byref(itc), ct.c_double(tau), ct.c_double(reg), int(ir_max),
                                ct.c_double(ir_tol), ct.byref(outc), ct.byref(kept))
    if rc != 0:
        raise ValueError(f"oracle Newton step failed (code {rc})")
    return out.view(), kept.value


def ir_residual(qp, iterate: dict, step: dict, rhs: dict) -> dict:
    """K*step + r for the Newton matrix K at `iterate` (Section 3.4)."""
    lib = _load()
    pk = _Packed(qp)
    it, st, rh, out = _vec_from(pk, iterate), _vec_from(pk, step), _vec_from(pk, rhs), Vec.like(pk)
    a, b, c, d = it.c(), st.c(), rh.c(), out.c()
    lib.orc_ir_residual(ct.byref(pk.c), ct.byref(a), ct.byref(b), ct.byref(c), ct.byref(d))
    return out.view()


def kkt_res(qp, sol: dict) -> float:
    """The KKT residual metric: max of the four residual inf-norms."""
    _, norms, _ = residuals(qp, sol)
    return float(np.max(norms))
