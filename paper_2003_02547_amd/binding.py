"""Thin Python binding of the C-ABI in include/oqp.h (liboqp.so).

Argument marshalling only: every step of the solver runs in the HIP kernels
of the library.  PyTorch provides the device buffer and the stream.  The
binding raises if the library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboqp.so")

OK, PENDING = 0, 1
EINVAL, ENOMEM, EDEVICE, EBUSY, ESTATE = -1, -2, -3, -4, -5
SUCCESS, MAX_ITER, MIN_STEP, NAN = 0, 1, 2, 3
MODE_F64, MODE_MIXED, MODE_ABS, MODE_ROBUST, MODE_BALANCE = 0, 1, 2, 3, 4

_P = ct.POINTER(ct.c_double)
_PI = ct.POINTER(ct.c_int)
_V = ct.c_void_p


class OqpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oqp error {code}: {msg}")
        self.code = code


class Arg(ct.Structure):
    _fields_ = [("mode", ct.c_int), ("tol_stat", ct.c_double), ("tol_eq", ct.c_double),
                ("tol_ineq", ct.c_double), ("tol_comp", ct.c_double), ("iter_max", ct.c_int),
                ("alpha_min", ct.c_double), ("gamma", ct.c_double), ("lam_min", ct.c_double),
                ("t_min", ct.c_double), ("reg_prim", ct.c_double), ("corr_ratio", ct.c_double),
                ("ir_max", ct.c_int), ("ir_tol", ct.c_double), ("warm_start", ct.c_int), ("cond_N", ct.c_int)]


class Stat(ct.Structure):
    _fields_ = [("status", ct.c_int), ("iters", ct.c_int), ("ir_steps", ct.c_int), ("fell_back_f64", ct.c_int),
                ("mu", ct.c_double), ("res", ct.c_double * 4), ("qr_refactors", ct.c_int)]


class ServerCfg(ct.Structure):
    _fields_ = [("max_requests", ct.c_int), ("max_launch", ct.c_int), ("max_groups", ct.c_int),
                ("staging_bytes", ct.c_size_t), ("iter_block", ct.c_int)]


class Counters(ct.Structure):
    _fields_ = [("submitted", ct.c_uint64), ("rejected", ct.c_uint64), ("completed", ct.c_uint64),
                ("launches", ct.c_uint64), ("queued", ct.c_int), ("running", ct.c_int), ("done", ct.c_int),
                ("dev_arena", ct.c_size_t), ("dev_used", ct.c_size_t), ("dev_peak", ct.c_size_t)]


_lib = None


def lib():
    """Load liboqp.so (built by build.build()); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2003_02547_amd.build.build()")
    # load torch's HIP runtime first so that the library binds to the same
    # one (device memory and streams come from torch)
    import torch  # noqa: F401
    L = ct.CDLL(LIB_PATH)
    sig = {
        "oqp_dims_bytes": (ct.c_size_t, [ct.c_int]),
        "oqp_dims_init": (ct.c_int, [_V, ct.c_size_t, ct.c_int, ct.POINTER(_V)]),
        "oqp_dims_set_stage": (ct.c_int, [_V, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int]),
        "oqp_dims_set_soft": (ct.c_int, [_V, ct.c_int, ct.c_int]),
        "oqp_qp_set_soft": (ct.c_int, [_V, ct.c_int, _PI, _P, _P, _P, _P, _P, _P]),
        "oqp_qp_get_soft": (ct.c_int, [_V, ct.c_int, _PI, _P, _P, _P, _P, _P, _P]),
        "oqp_batch_get_soft_sol": (ct.c_int, [_V, ct.c_int, _P, _P, _P, _P, _P, _P]),
        "oqp_batch_set_soft_iterate": (ct.c_int, [_V, ct.c_int, _P, _P, _P, _P, _P, _P]),
        "oqp_batch_get_soft_step": (ct.c_int, [_V, ct.c_int, _P, _P, _P, _P, _P, _P]),
        "oqp_batch_nsoft": (ct.c_int, [_V, ct.c_int]),
        "oqp_server_get_soft_sol": (ct.c_int, [_V, ct.c_uint64, _P, _P, _P, _P, _P, _P]),
        "oqp_qp_bytes": (ct.c_size_t, [_V]),
        "oqp_qp_init": (ct.c_int, [_V, _V, ct.c_size_t, ct.POINTER(_V)]),
        "oqp_qp_set_dyn": (ct.c_int, [_V, ct.c_int, _P, ct.c_int, _P, ct.c_int, _P]),
        "oqp_qp_set_cost": (ct.c_int, [_V, ct.c_int, _P, ct.c_int, _P, ct.c_int, _P, ct.c_int, _P, _P]),
        "oqp_qp_set_box_u": (ct.c_int, [_V, ct.c_int, _PI, _P, _P]),
        "oqp_qp_set_box_x": (ct.c_int, [_V, ct.c_int, _PI, _P, _P]),
        "oqp_qp_set_general": (ct.c_int, [_V, ct.c_int, _P, ct.c_int, _P, ct.c_int, _P, _P]),
        "oqp_qp_get_dyn": (ct.c_int, [_V, ct.c_int, _P, ct.c_int, _P, ct.c_int, _P]),
        "oqp_qp_get_cost": (ct.c_int, [_V, ct.c_int, _P, ct.c_int, _P, ct.c_int, _P, ct.c_int, _P, _P]),
        "oqp_qp_get_box_u": (ct.c_int, [_V, ct.c_int, _PI, _P, _P]),
        "oqp_qp_get_box_x": (ct.c_int, [_V, ct.c_int, _PI, _P, _P]),
        "oqp_qp_get_general": (ct.c_int, [_V, ct.c_int, _P, ct.c_int, _P, ct.c_int, _P, _P]),
        "oqp_pcond_dims_bytes": (ct.c_size_t, [_V, ct.c_int]),
        "oqp_pcond_dims": (ct.c_int, [_V, ct.c_int, _V, ct.c_size_t, ct.POINTER(_V)]),
        "oqp_batch_fetch_cond": (ct.c_int, [_V]),
        "oqp_batch_set_streams": (ct.c_int, [_V, ct.POINTER(_V), ct.c_int]),
        "oqp_batch_init_static": (ct.c_int, [ct.POINTER(_V), ct.c_int, ct.POINTER(Arg), _V, ct.c_size_t, _V,
                                             ct.POINTER(_V)]),
        "oqp_set_variant_mask": (ct.c_int, [ct.c_uint]),
        "oqp_get_variant_mask": (ct.c_uint, []),
        "oqp_set_lds_split": (ct.c_int, [ct.c_int]),
        "oqp_get_lds_split": (ct.c_int, []),
        "oqp_batch_release": (ct.c_int, [_V]),
        "oqp_batch_get_cond_qp": (ct.c_int, [_V, ct.c_int, _V]),
        "oqp_arg_default": (None, [ct.POINTER(Arg), ct.c_int]),
        "oqp_batch_bytes": (ct.c_int, [ct.POINTER(_V), ct.c_int, ct.POINTER(Arg), ct.POINTER(ct.c_size_t),
                                       ct.POINTER(ct.c_size_t)]),
        "oqp_batch_init": (ct.c_int, [ct.POINTER(_V), ct.c_int, ct.POINTER(Arg), _V, ct.c_size_t, _V, ct.c_size_t,
                                      _V, ct.POINTER(_V)]),
        "oqp_batch_load": (ct.c_int, [_V, ct.POINTER(_V)]),
        "oqp_batch_solve": (ct.c_int, [_V]),
        "oqp_batch_set_arg": (ct.c_int, [_V, ct.POINTER(Arg)]),
        "oqp_batch_fetch": (ct.c_int, [_V]),
        "oqp_batch_sync": (ct.c_int, [_V]),
        "oqp_batch_get_stat": (ct.c_int, [_V, ct.c_int, ct.POINTER(Stat)]),
        "oqp_batch_get_sol": (ct.c_int, [_V, ct.c_int, _P, _P, _P, _P, _P, _P, _P]),
        "oqp_batch_set_iterate": (ct.c_int, [_V, ct.c_int, _P, _P, _P, _P, _P, _P, _P]),
        "oqp_batch_newton": (ct.c_int, [_V, ct.c_double]),
        "oqp_batch_get_step": (ct.c_int, [_V, ct.c_int, _P, _P, _P, _P, _P, _P, _P]),
        "oqp_batch_variant": (ct.c_int, [_V, ct.c_int, _PI, _PI, _PI]),
        "oqp_pack_bytes": (ct.c_int, [_V, ct.POINTER(ct.c_size_t)]),
        "oqp_pack": (ct.c_int, [_V, _V, ct.c_size_t]),
        "oqp_pack_footprint": (ct.c_int, [_V, ct.POINTER(ct.c_size_t), _PI]),
        "oqp_server_cfg_default": (None, [ct.POINTER(ServerCfg)]),
        "oqp_server_bytes": (ct.c_int, [ct.POINTER(ServerCfg), ct.POINTER(ct.c_size_t), ct.POINTER(ct.c_size_t)]),
        "oqp_server_init": (ct.c_int, [ct.POINTER(ServerCfg), ct.POINTER(Arg), _V, ct.c_size_t, _V, ct.c_size_t,
                                       ct.POINTER(_V), ct.c_int, ct.POINTER(_V)]),
        "oqp_server_destroy": (ct.c_int, [_V]),
        "oqp_server_submit": (ct.c_int, [_V, _V, ct.POINTER(ct.c_uint64)]),
        "oqp_server_progress": (ct.c_int, [_V, _PI]),
        "oqp_server_poll": (ct.c_int, [_V, ct.c_uint64, ct.POINTER(Stat)]),
        "oqp_server_latency": (ct.c_int, [_V, ct.c_uint64, _P]),
        "oqp_server_get_sol": (ct.c_int, [_V, ct.c_uint64, _P, _P, _P, _P, _P, _P, _P]),
        "oqp_server_release": (ct.c_int, [_V, ct.c_uint64]),
        "oqp_server_stats": (ct.c_int, [_V, ct.POINTER(Counters)]),
        "oqp_server_replay": (ct.c_int, [_V, ct.POINTER(_V), _P, ct.c_int, ct.c_double, _P, ct.POINTER(Stat), _P]),
        "oqp_sol_bytes": (ct.c_size_t, [_V]),
        "oqp_sol_init": (ct.c_int, [_V, _V, ct.c_size_t, ct.POINTER(_V)]),
        "oqp_batch_fill_sol": (ct.c_int, [_V, ct.c_int, _V]),
        "oqp_server_fill_sol": (ct.c_int, [_V, ct.c_uint64, _V]),
        "oqp_sol_get_stat": (ct.c_int, [_V, ct.POINTER(Stat)]),
        "oqp_res_get_norms": (ct.c_int, [_V, _P]),
        "oqp_sol_get_u": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_x": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_pi": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_lam_lb_u": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_lam_ub_u": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_lam_lb_x": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_lam_ub_x": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_lam_lg": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_lam_ug": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_t_lb_u": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_t_ub_u": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_t_lb_x": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_t_ub_x": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_t_lg": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_sol_get_t_ug": (ct.c_int, [_V, ct.c_int, _P]),
        "oqp_set_wave_max": (ct.c_int, [ct.c_int]),
        "oqp_get_wave_max": (ct.c_int, []),
        "oqp_variant_count": (ct.c_int, []),
        "oqp_variant_dims": (ct.c_int, [ct.c_int, _PI, _PI, _PI]),
        "oqp_last_error": (ct.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc):
    if rc < 0:
        raise OqpError(rc, lib().oqp_last_error().decode())
    return rc


def _aligned(nbytes: int, align: int = 64) -> np.ndarray:
    raw = np.zeros(nbytes + align, dtype=np.uint8)
    off = (-raw.ctypes.data) % align
    return raw[off:off + nbytes]


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(_P)


def _f64(a, shape=None):
    a = np.asarray(a, dtype=np.float64)
    return np.asfortranarray(a)


def default_arg(mode: int = MODE_F64, **overrides) -> Arg:
    a = Arg()
    lib().oqp_arg_default(ct.byref(a), mode)
    for k, v in overrides.items():
        setattr(a, k, v)
    return a


class _DimsC(ct.Structure):
    _fields_ = [("N", ct.c_int)] + [(k, ct.POINTER(ct.c_int)) for k in ("nx", "nu", "nbu", "nbx", "ng", "ns")]


SOFT_FIELDS = ("Zl", "Zu", "zl", "zu", "lls", "lus")
SOFT_KEYS = ("s_l", "s_u", "lam_sl", "lam_su", "t_sl", "t_su")


def _has_soft(qp) -> bool:
    return getattr(qp, "idxs", None) is not None and any(len(i) for i in qp.idxs)


class Dims:
    def __init__(self, N: int, nx, nu, nbu, nbx, ng, ns=None):
        L = lib()
        self.N = N
        self.mem = _aligned(L.oqp_dims_bytes(N))
        h = _V()
        _check(L.oqp_dims_init(self.mem.ctypes.data, self.mem.nbytes, N, ct.byref(h)))
        self.h = h
        for n in range(N + 1):
            _check(L.oqp_dims_set_stage(h, n, int(nx[n]), int(nu[n]), int(nbu[n]), int(nbx[n]), int(ng[n])))
            if ns is not None:
                _check(L.oqp_dims_set_soft(h, n, int(ns[n])))

    @classmethod
    def of(cls, qp) -> "Dims":
        ns = [len(i) for i in qp.idxs] if getattr(qp, "idxs", None) is not None else None
        return cls(qp.N, qp.nx, qp.nu, qp.nbu, qp.nbx, qp.ng, ns)

    @classmethod
    def condensed(cls, qp, cond_N: int) -> "Dims":
        """Dims of the partially condensed QP (oqp_pcond_dims)."""
        L = lib()
        src = Dims.of(qp)
        mem = _aligned(L.oqp_pcond_dims_bytes(src.h, int(cond_N)))
        h = _V()
        _check(L.oqp_pcond_dims(src.h, int(cond_N), mem.ctypes.data, mem.nbytes, ct.byref(h)))
        c = ct.cast(h, ct.POINTER(_DimsC)).contents
        N = c.N
        sizes = {k: [getattr(c, k)[n] for n in range(N + 1)] for k in ("nx", "nu", "nbu", "nbx", "ng")}
        return cls(N, **sizes)

    def sizes(self):
        c = ct.cast(self.h, ct.POINTER(_DimsC)).contents
        return {k: [getattr(c, k)[n] for n in range(self.N + 1)] for k in ("nx", "nu", "nbu", "nbx", "ng", "ns")}


class Qp:
    """oqp_qp built from an OcpQp-like object through the per-stage setters."""

    def __init__(self, qp, dims: Dims | None = None):
        L = lib()
        self.dims = dims or Dims.of(qp)
        self.mem = _aligned(L.oqp_qp_bytes(self.dims.h))
        h = _V()
        _check(L.oqp_qp_init(self.dims.h, self.mem.ctypes.data, self.mem.nbytes, ct.byref(h)))
        self.h = h
        N = qp.N
        for n in range(N + 1):
            nx, nu = qp.nx[n], qp.nu[n]
            if n < N:
                A, B, b = _f64(qp.A[n]), _f64(qp.B[n]), _f64(qp.b[n])
                _check(L.oqp_qp_set_dyn(h, n, _p(A), max(A.shape[0], 1), _p(B), max(B.shape[0], 1), _p(b)))
            Q, S, R = _f64(qp.Q[n]), _f64(qp.S[n]), _f64(qp.R[n])
            q, r = _f64(qp.q[n]), _f64(qp.r[n])
            _check(L.oqp_qp_set_cost(h, n, _p(Q), max(nx, 1), _p(S), max(nu, 1), _p(R), max(nu, 1), _p(q), _p(r)))
            if len(qp.idxbu[n]):
                iu = np.ascontiguousarray(qp.idxbu[n], dtype=np.int32)
                _check(L.oqp_qp_set_box_u(h, n, iu.ctypes.data_as(_PI), _p(_f64(qp.lbu[n])), _p(_f64(qp.ubu[n]))))
            if len(qp.idxbx[n]):
                ix = np.ascontiguousarray(qp.idxbx[n], dtype=np.int32)
                _check(L.oqp_qp_set_box_x(h, n, ix.ctypes.data_as(_PI), _p(_f64(qp.lbx[n])), _p(_f64(qp.ubx[n]))))
            ng = np.asarray(qp.D[n]).shape[0]
            if ng:
                D, C = _f64(qp.D[n]), _f64(qp.C[n])
                _check(L.oqp_qp_set_general(h, n, _p(D), ng, _p(C), ng, _p(_f64(qp.lg[n])), _p(_f64(qp.ug[n]))))
            if getattr(qp, "idxs", None) is not None and len(qp.idxs[n]):
                js = np.ascontiguousarray(qp.idxs[n], dtype=np.int32)
                vals = [_f64(getattr(qp, k)[n]) for k in SOFT_FIELDS]
                _check(L.oqp_qp_set_soft(h, n, js.ctypes.data_as(_PI), *[_p(v) for v in vals]))


@dataclass
class Result:
    status: int
    iters: int
    ir_steps: int
    mu: float
    res: np.ndarray
    sol: dict
    fell_back_f64: int = 0
    qr_refactors: int = 0


def _sizes(qp):
    return (int(sum(qp.nu)), int(sum(qp.nx)), int(sum(qp.nx[1:])), int(qp.n_constraints()))


class Batch:
    """A batch of OCP QPs solved on the current CUDA (HIP) device and stream."""

    def __init__(self, qps: Sequence, arg: Arg | None = None, device=None, stream=None, streams=0,
                 static: bool = False):
        """streams: extra streams for concurrent kernel groups, a count (new
        default-priority streams) or a list of existing torch streams (a
        caller that keeps a fixed set of streams controls which hardware
        queues they share).  static=True: the batch's device records go to the
        library's static device region (oqp_batch_init_static) instead of a
        device buffer allocated here; one such batch at a time per GPU, no
        extra streams."""
        import torch
        L = lib()
        self.qps = list(qps)
        self.arg = arg or default_arg()
        self.dims = [Dims.of(q) for q in self.qps]
        n = len(self.qps)
        self._dimh = (_V * n)(*[d.h for d in self.dims])
        hb, db = ct.c_size_t(0), ct.c_size_t(0)
        _check(L.oqp_batch_bytes(self._dimh, n, ct.byref(self.arg), ct.byref(hb), ct.byref(db)))
        self.host_bytes, self.dev_bytes = hb.value, db.value
        self.host = _aligned(self.host_bytes, 64)
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = _V()
        if static:
            if streams:
                raise ValueError("a batch in the static device region takes no extra streams")
            self.dev_buf, self.dev_ptr = None, None
            with torch.cuda.device(dev):
                _check(L.oqp_batch_init_static(self._dimh, n, ct.byref(self.arg), self.host.ctypes.data,
                                               self.host_bytes, self.stream.cuda_stream, ct.byref(h)))
        else:
            self.dev_buf = torch.empty(self.dev_bytes + 256, dtype=torch.uint8, device=dev)
            base = self.dev_buf.data_ptr()
            self.dev_ptr = base + ((-base) % 256)
            _check(L.oqp_batch_init(self._dimh, n, ct.byref(self.arg), self.host.ctypes.data, self.host_bytes,
                                    self.dev_ptr, self.dev_bytes, self.stream.cuda_stream, ct.byref(h)))
        self.h = h
        self._qph = None
        self.aux = []
        if isinstance(streams, (list, tuple)):
            self.aux = list(streams)
        elif streams > 0:
            # extra streams (default priority) for concurrent kernel groups
            self.aux = [torch.cuda.Stream(device=dev) for _ in range(int(streams))]
        if self.aux:
            arr = (_V * len(self.aux))(*[s.cuda_stream for s in self.aux])
            _check(L.oqp_batch_set_streams(self.h, arr, len(self.aux)))

    def __del__(self):
        try:
            if getattr(self, "aux", None) and self.h:
                lib().oqp_batch_release(self.h)
        except Exception:
            pass

    def load(self):
        L = lib()
        self._qpo = [Qp(q, d) for q, d in zip(self.qps, self.dims)]
        self._qph = (_V * len(self._qpo))(*[q.h for q in self._qpo])
        _check(L.oqp_batch_load(self.h, self._qph))
        return self

    def solve(self):
        _check(lib().oqp_batch_solve(self.h))
        return self

    def set_arg(self, arg: Arg):
        _check(lib().oqp_batch_set_arg(self.h, ct.byref(arg)))
        self.arg = arg

    def fetch(self):
        _check(lib().oqp_batch_fetch(self.h))
        return self

    def sync(self):
        _check(lib().oqp_batch_sync(self.h))
        return self

    def stat(self, i: int) -> Stat:
        st = Stat()
        _check(lib().oqp_batch_get_stat(self.h, i, ct.byref(st)))
        return st

    def _alloc_vec(self, i):
        nu, nx, npi, nc = _sizes(self.qps[i])
        return {k: np.zeros(max(s, 1)) for k, s in
                (("u", nu), ("x", nx), ("pi", npi), ("lam_l", nc), ("lam_u", nc), ("t_l", nc), ("t_u", nc))}, \
            dict(u=nu, x=nx, pi=npi, lam_l=nc, lam_u=nc, t_l=nc, t_u=nc)

    def _soft_vec(self, i):
        ns = int(sum(len(j) for j in self.qps[i].idxs)) if _has_soft(self.qps[i]) else 0
        return ns, {k: np.zeros(max(ns, 1)) for k in SOFT_KEYS}

    def solution(self, i: int) -> dict:
        v, sz = self._alloc_vec(i)
        _check(lib().oqp_batch_get_sol(self.h, i, *[_p(v[k]) for k in ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u")]))
        out = {k: v[k][:sz[k]].copy() for k in v}
        if _has_soft(self.qps[i]):
            ns, sv = self._soft_vec(i)
            _check(lib().oqp_batch_get_soft_sol(self.h, i, *[_p(sv[k]) for k in SOFT_KEYS]))
            out.update({k: sv[k][:ns].copy() for k in SOFT_KEYS})
        return out

    def result(self, i: int) -> Result:
        st = self.stat(i)
        return Result(st.status, st.iters, st.ir_steps, st.mu, np.array(st.res[:]), self.solution(i), st.fell_back_f64,
                      st.qr_refactors)

    def results(self) -> List[Result]:
        return [self.result(i) for i in range(len(self.qps))]

    def set_iterate(self, i: int, it: dict):
        v, sz = self._alloc_vec(i)
        for k in v:
            v[k][:sz[k]] = np.asarray(it[k], dtype=np.float64)[:sz[k]]
        _check(lib().oqp_batch_set_iterate(self.h, i, *[_p(v[k]) for k in ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u")]))
        if _has_soft(self.qps[i]):
            ns, sv = self._soft_vec(i)
            for k in SOFT_KEYS:
                sv[k][:ns] = np.asarray(it[k], dtype=np.float64)[:ns]
            _check(lib().oqp_batch_set_soft_iterate(self.h, i, *[_p(sv[k]) for k in SOFT_KEYS]))

    def newton(self, tau: float = 0.0):
        _check(lib().oqp_batch_newton(self.h, ct.c_double(tau)))
        return self

    def step(self, i: int) -> dict:
        v, sz = self._alloc_vec(i)
        _check(lib().oqp_batch_get_step(self.h, i, *[_p(v[k]) for k in ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u")]))
        out = {k: v[k][:sz[k]].copy() for k in v}
        if _has_soft(self.qps[i]):
            ns, sv = self._soft_vec(i)
            _check(lib().oqp_batch_get_soft_step(self.h, i, *[_p(sv[k]) for k in SOFT_KEYS]))
            out.update({k: sv[k][:ns].copy() for k in SOFT_KEYS})
        return out

    def variant(self, i: int):
        a, b, c = ct.c_int(), ct.c_int(), ct.c_int()
        v = lib().oqp_batch_variant(self.h, i, ct.byref(a), ct.byref(b), ct.byref(c))
        return v, (a.value, b.value, c.value)

    def fetch_cond(self):
        _check(lib().oqp_batch_fetch_cond(self.h))
        return self

    def cond_qp(self, i: int):
        """The condensed QP of instance i (after fetch_cond + sync), with the
        field names of an OcpQp."""
        d = Dims.condensed(self.qps[i], self.arg.cond_N)
        L = lib()
        mem = _aligned(L.oqp_qp_bytes(d.h))
        h = _V()
        _check(L.oqp_qp_init(d.h, mem.ctypes.data, mem.nbytes, ct.byref(h)))
        _check(L.oqp_batch_get_cond_qp(self.h, i, h))
        return qp_fields(h, d)


def qp_fields(h, dims: Dims):
    """Read an oqp_qp back through the getters into OcpQp field lists."""
    L = lib()
    sz = dims.sizes()
    N = dims.N
    out = {k: [] for k in ("A", "B", "b", "Q", "S", "R", "q", "r", "idxbu", "lbu", "ubu", "idxbx", "lbx", "ubx",
                           "D", "C", "lg", "ug")}
    for n in range(N + 1):
        nx, nu, nbu, nbx, ng = (sz[k][n] for k in ("nx", "nu", "nbu", "nbx", "ng"))
        if n < N:
            nxn = sz["nx"][n + 1]
            A, B, b = np.zeros((nxn, nx), order="F"), np.zeros((nxn, nu), order="F"), np.zeros(nxn)
            _check(L.oqp_qp_get_dyn(h, n, _p(A), max(nxn, 1), _p(B), max(nxn, 1), _p(b)))
            out["A"].append(A); out["B"].append(B); out["b"].append(b)
        Q, S, R = np.zeros((nx, nx), order="F"), np.zeros((nu, nx), order="F"), np.zeros((nu, nu), order="F")
        q, r = np.zeros(nx), np.zeros(nu)
        _check(L.oqp_qp_get_cost(h, n, _p(Q), max(nx, 1), _p(S), max(nu, 1), _p(R), max(nu, 1), _p(q), _p(r)))
        out["Q"].append(Q); out["S"].append(S); out["R"].append(R); out["q"].append(q); out["r"].append(r)
        for key, nb, fn in (("u", nbu, L.oqp_qp_get_box_u), ("x", nbx, L.oqp_qp_get_box_x)):
            idx, lo, hi = np.zeros(max(nb, 1), dtype=np.int32), np.zeros(max(nb, 1)), np.zeros(max(nb, 1))
            _check(fn(h, n, idx.ctypes.data_as(_PI), _p(lo), _p(hi)))
            out["idxb" + key].append(idx[:nb].copy()); out["lb" + key].append(lo[:nb].copy())
            out["ub" + key].append(hi[:nb].copy())
        D, C = np.zeros((ng, nu), order="F"), np.zeros((ng, nx), order="F")
        lg, ug = np.zeros(max(ng, 1)), np.zeros(max(ng, 1))
        _check(L.oqp_qp_get_general(h, n, _p(D), max(ng, 1), _p(C), max(ng, 1), _p(lg), _p(ug)))
        out["D"].append(D); out["C"].append(C); out["lg"].append(lg[:ng].copy()); out["ug"].append(ug[:ng].copy())
        ns = sz["ns"][n]
        js = np.zeros(max(ns, 1), dtype=np.int32)
        sv = [np.zeros(max(ns, 1)) for _ in SOFT_FIELDS]
        _check(L.oqp_qp_get_soft(h, n, js.ctypes.data_as(_PI), *[_p(v) for v in sv]))
        out.setdefault("idxs", []).append(js[:ns].copy())
        for k, v in zip(SOFT_FIELDS, sv):
            out.setdefault(k, []).append(v[:ns].copy())
    import types
    return types.SimpleNamespace(N=N, nx=sz["nx"], nu=sz["nu"], **out)


def solve(qps: Sequence, arg: Arg | None = None) -> List[Result]:
    """Load, solve, fetch and return the results of a batch."""
    b = Batch(qps, arg).load().solve().fetch().sync()
    return b.results()


_KEYS = ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u")

SOL_FIELDS = ("u", "x", "pi", "lam_lb_u", "lam_ub_u", "lam_lb_x", "lam_ub_x", "lam_lg", "lam_ug", "t_lb_u", "t_ub_u",
              "t_lb_x", "t_ub_x", "t_lg", "t_ug")


class Sol:
    """oqp_sol in caller memory with the per-stage getters."""

    def __init__(self, dims: "Dims"):
        L = lib()
        self.dims = dims
        self.mem = _aligned(L.oqp_sol_bytes(dims.h), 64)
        h = _V()
        _check(L.oqp_sol_init(dims.h, self.mem.ctypes.data, self.mem.nbytes, ct.byref(h)))
        self.h = h

    def fill_from_batch(self, batch: "Batch", i: int):
        _check(lib().oqp_batch_fill_sol(batch.h, i, self.h))
        return self

    def fill_from_server(self, server: "Server", ticket: int):
        _check(lib().oqp_server_fill_sol(server.h, ticket, self.h))
        return self

    def get(self, field: str, n: int, size: int) -> np.ndarray:
        out = np.zeros(max(size, 1))
        _check(getattr(lib(), "oqp_sol_get_" + field)(self.h, n, _p(out)))
        return out[:size].copy()

    def norms(self) -> np.ndarray:
        out = np.zeros(4)
        _check(lib().oqp_res_get_norms(self.h, _p(out)))
        return out


def _sol_buffers(qp):
    nu, nx, npi, nc = _sizes(qp)
    sz = dict(u=nu, x=nx, pi=npi, lam_l=nc, lam_u=nc, t_l=nc, t_u=nc)
    return {k: np.zeros(max(sz[k], 1)) for k in _KEYS}, sz


class Packed:
    """A QP packed once into the relocatable request blob (oqp_pack).

    pinned=True places the blob in page-locked host memory (a pinned torch
    tensor) so that the server's uploads are asynchronous DMA copies."""

    def __init__(self, qp, pinned: bool = False):
        L = lib()
        self.qp = qp
        q = Qp(qp)
        nb = ct.c_size_t()
        _check(L.oqp_pack_bytes(q.h, ct.byref(nb)))
        self.nbytes = nb.value
        if pinned:
            import torch
            self._mem = torch.empty(self.nbytes + 64, dtype=torch.uint8, pin_memory=True)
            base = self._mem.data_ptr()
        else:
            self._mem = np.zeros(self.nbytes + 64, dtype=np.uint8)
            base = self._mem.ctypes.data
        self.ptr = base + ((-base) % 64)
        _check(L.oqp_pack(q.h, self.ptr, self.nbytes))
        fb, v = ct.c_size_t(), ct.c_int()
        _check(L.oqp_pack_footprint(self.ptr, ct.byref(fb), ct.byref(v)))
        self.footprint, self.variant = fb.value, v.value


class Server:
    """Continuous-batching server on the current device (oqp_server_*).

    Streams are created here with the default priority; the server's host
    memory is a pinned torch tensor, its device arena a byte tensor."""

    def __init__(self, arg: Arg | None = None, dev_bytes: int = 1 << 30, nstreams: int = 8, device=None, **cfg):
        import torch
        L = lib()
        self.arg = arg or default_arg()
        c = ServerCfg()
        L.oqp_server_cfg_default(ct.byref(c))
        for k, v in cfg.items():
            setattr(c, k, v)
        self.cfg = c
        hb, fb = ct.c_size_t(), ct.c_size_t()
        _check(L.oqp_server_bytes(ct.byref(c), ct.byref(hb), ct.byref(fb)))
        self.host_bytes = hb.value
        self.dev_bytes = int(dev_bytes) + fb.value
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._host = torch.empty(self.host_bytes + 64, dtype=torch.uint8, pin_memory=True)
        hp = self._host.data_ptr() + ((-self._host.data_ptr()) % 64)
        self._dev = torch.empty(self.dev_bytes + 256, dtype=torch.uint8, device=dev)
        dp = self._dev.data_ptr() + ((-self._dev.data_ptr()) % 256)
        self.streams = [torch.cuda.Stream(dev) for _ in range(nstreams)]
        self._sh = (_V * nstreams)(*[st.cuda_stream for st in self.streams])
        h = _V()
        _check(L.oqp_server_init(ct.byref(c), ct.byref(self.arg), hp, self.host_bytes, dp, self.dev_bytes, self._sh,
                                 nstreams, ct.byref(h)))
        self.h = h
        self._tickets = {}

    def submit(self, packed: Packed):
        """Ticket, or None when admission is refused (OQP_EBUSY)."""
        t = ct.c_uint64()
        rc = lib().oqp_server_submit(self.h, packed.ptr, ct.byref(t))
        if rc == EBUSY:
            return None
        _check(rc)
        self._tickets[t.value] = packed
        return t.value

    def progress(self) -> int:
        n = ct.c_int()
        _check(lib().oqp_server_progress(self.h, ct.byref(n)))
        return n.value

    def poll(self, ticket):
        st = Stat()
        rc = _check(lib().oqp_server_poll(self.h, ticket, ct.byref(st)))
        return None if rc == PENDING else st

    def latency(self, ticket) -> float:
        v = ct.c_double()
        _check(lib().oqp_server_latency(self.h, ticket, ct.byref(v)))
        return v.value

    def solution(self, ticket) -> dict:
        qp = self._tickets[ticket].qp
        v, sz = _sol_buffers(qp)
        _check(lib().oqp_server_get_sol(self.h, ticket, *[_p(v[k]) for k in _KEYS]))
        out = {k: v[k][:sz[k]].copy() for k in _KEYS}
        if _has_soft(qp):
            ns = int(sum(len(j) for j in qp.idxs))
            sv = {k: np.zeros(max(ns, 1)) for k in SOFT_KEYS}
            _check(lib().oqp_server_get_soft_sol(self.h, ticket, *[_p(sv[k]) for k in SOFT_KEYS]))
            out.update({k: sv[k][:ns].copy() for k in SOFT_KEYS})
        return out

    def result(self, ticket) -> Result:
        st = self.poll(ticket)
        return Result(st.status, st.iters, st.ir_steps, st.mu, np.array(st.res[:]), self.solution(ticket),
                      st.fell_back_f64, st.qr_refactors)

    def release(self, ticket):
        _check(lib().oqp_server_release(self.h, ticket))
        self._tickets.pop(ticket, None)

    def stats(self) -> dict:
        c = Counters()
        _check(lib().oqp_server_stats(self.h, ct.byref(c)))
        return {k: getattr(c, k) for k, _ in Counters._fields_}

    def replay(self, packed: Sequence[Packed], arrival, timeout: float = 60.0):
        """Native real-time replay of an arrival schedule; returns
        (latency seconds, per-request Stat list, wall seconds)."""
        n = len(packed)
        arr = np.ascontiguousarray(arrival, dtype=np.float64)
        ptrs = (_V * n)(*[p.ptr for p in packed])
        lat = np.zeros(max(n, 1))
        stats = (Stat * max(n, 1))()
        wall = ct.c_double()
        _check(lib().oqp_server_replay(self.h, ptrs, _p(arr), n, ct.c_double(timeout), _p(lat), stats,
                                       ct.byref(wall)))
        return lat[:n], list(stats)[:n], wall.value

    def close(self):
        if self.h:
            _check(lib().oqp_server_destroy(self.h))
            self.h = None

    def __del__(self):
        # oqp_server_destroy waits for the server's streams and destroys its
        # events before the arena and host tensors are released, so a server
        # dropped without close() leaves no launch reading freed memory
        try:
            if getattr(self, "h", None):
                lib().oqp_server_destroy(self.h)
                self.h = None
        except Exception:
            pass


def set_wave_max(nz: int) -> int:
    """Largest stage block (nx + nu, padded) solved by the one-wave kernels;
    larger instances go to the block kernel.  Returns the previous bound."""
    L = lib()
    old = L.oqp_get_wave_max()
    _check(L.oqp_set_wave_max(int(nz)))
    return old


def variants():
    L = lib()
    out = []
    for v in range(L.oqp_variant_count()):
        a, b, c = ct.c_int(), ct.c_int(), ct.c_int()
        L.oqp_variant_dims(v, ct.byref(a), ct.byref(b), ct.byref(c))
        out.append((a.value, b.value, c.value))
    return out


EXPORTED = [
    "oqp_dims_bytes", "oqp_dims_init", "oqp_dims_set_stage", "oqp_qp_bytes", "oqp_qp_init", "oqp_qp_set_dyn",
    "oqp_qp_set_cost", "oqp_qp_set_box_u", "oqp_qp_set_box_x", "oqp_qp_set_general", "oqp_arg_default",
    "oqp_batch_bytes", "oqp_batch_init", "oqp_batch_load", "oqp_batch_solve", "oqp_batch_set_arg",
    "oqp_batch_fetch", "oqp_batch_sync", "oqp_batch_get_stat", "oqp_batch_get_sol", "oqp_batch_set_iterate",
    "oqp_batch_newton", "oqp_batch_get_step", "oqp_batch_variant", "oqp_variant_count", "oqp_variant_dims",
    "oqp_last_error", "oqp_pack_bytes", "oqp_pack", "oqp_pack_footprint", "oqp_server_cfg_default",
    "oqp_server_bytes", "oqp_server_init", "oqp_server_destroy", "oqp_server_submit", "oqp_server_progress",
    "oqp_server_poll", "oqp_server_latency", "oqp_server_get_sol", "oqp_server_release", "oqp_server_stats",
    "oqp_server_replay", "oqp_set_wave_max", "oqp_get_wave_max", "oqp_sol_bytes", "oqp_sol_init",
    "oqp_batch_fill_sol", "oqp_server_fill_sol", "oqp_sol_get_stat", "oqp_res_get_norms",
    "oqp_qp_get_dyn", "oqp_qp_get_cost", "oqp_qp_get_box_u", "oqp_qp_get_box_x", "oqp_qp_get_general",
    "oqp_pcond_dims_bytes", "oqp_pcond_dims", "oqp_batch_fetch_cond", "oqp_batch_get_cond_qp",
    "oqp_batch_set_streams", "oqp_batch_release", "oqp_dims_set_soft", "oqp_qp_set_soft", "oqp_qp_get_soft",
    "oqp_batch_get_soft_sol", "oqp_batch_set_soft_iterate", "oqp_batch_get_soft_step", "oqp_batch_nsoft",
    "oqp_server_get_soft_sol", "oqp_batch_init_static", "oqp_set_variant_mask", "oqp_get_variant_mask",
    "oqp_set_lds_split", "oqp_get_lds_split",
] + ["oqp_sol_get_" + g for g in SOL_FIELDS]
