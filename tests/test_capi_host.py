"""Host-side checks of the C-ABI (no GPU needed): the library loads, exports
every function include/oqp.h declares, and rejects bad input before any
device call."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

from paper_2003_02547_amd import binding as B
from paper_2003_02547_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "oqp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(oqp_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.EXPORTED)


def test_variant_table():
    v = B.variants()
    assert (16, 8, 0) in v and (8, 4, 0) in v
    for nx, nu, ng in v:
        assert nx + nu <= 64 and ng <= 64


def test_dims_errors():
    L = B.lib()
    assert L.oqp_dims_bytes(0) == 0
    mem = B._aligned(L.oqp_dims_bytes(3))
    h = ct.c_void_p()
    assert L.oqp_dims_init(mem.ctypes.data, 8, 3, ct.byref(h)) == B.ENOMEM
    assert L.oqp_dims_init(mem.ctypes.data, mem.nbytes, 0, ct.byref(h)) == B.EINVAL
    assert L.oqp_dims_init(mem.ctypes.data, mem.nbytes, 3, ct.byref(h)) == B.OK
    assert L.oqp_dims_set_stage(h, 4, 1, 1, 0, 0, 0) == B.EINVAL
    assert L.oqp_dims_set_stage(h, 1, 2, 1, 2, 0, 0) == B.EINVAL  # nbu > nu
    assert L.oqp_dims_set_stage(h, 1, 2, 1, 1, 2, 0) == B.OK
    assert b"oqp_dims_set_stage" in L.oqp_last_error() or L.oqp_last_error() is not None


def test_qp_setter_errors():
    qp = W.mass_spring_chain4(1)
    q = B.Qp(qp)
    L = B.lib()
    idx = np.array([0, 0, 1], dtype=np.int32)
    lo = np.zeros(3); hi = np.ones(3)
    rc = L.oqp_qp_set_box_u(q.h, 0, idx.ctypes.data_as(B._PI), B._p(lo), B._p(hi))
    assert rc == B.EINVAL and b"repeated" in L.oqp_last_error()
    idx = np.array([0, 1, 5], dtype=np.int32)
    rc = L.oqp_qp_set_box_u(q.h, 0, idx.ctypes.data_as(B._PI), B._p(lo), B._p(hi))
    assert rc == B.EINVAL
    idx = np.array([0, 1, 2], dtype=np.int32)
    rc = L.oqp_qp_set_box_u(q.h, 0, idx.ctypes.data_as(B._PI), B._p(hi), B._p(lo))
    assert rc == B.EINVAL and b"lo > hi" in L.oqp_last_error()
    A = np.eye(8)
    assert L.oqp_qp_set_dyn(q.h, 10, B._p(A), 8, None, 8, None) == B.EINVAL  # stage N has no dynamics
    assert L.oqp_qp_set_dyn(q.h, 0, B._p(A), 4, None, 8, None) == B.EINVAL   # lda too small


def test_batch_size_and_plan_errors():
    L = B.lib()
    arg = B.default_arg()
    qps = [W.mass_spring_chain4(s) for s in range(3)]
    dims = [B.Dims.of(q) for q in qps]
    arr = (ct.c_void_p * 3)(*[d.h for d in dims])
    hb, db = ct.c_size_t(), ct.c_size_t()
    assert L.oqp_batch_bytes(arr, 3, ct.byref(arg), ct.byref(hb), ct.byref(db)) == B.OK
    assert hb.value > 0 and db.value > 0
    # too small buffers are refused before any device call
    host = B._aligned(hb.value)
    h = ct.c_void_p()
    rc = L.oqp_batch_init(arr, 3, ct.byref(arg), host.ctypes.data, hb.value, ct.c_void_p(256), db.value - 1,
                          None, ct.byref(h))
    assert rc == B.ENOMEM
    rc = L.oqp_batch_init(arr, 3, ct.byref(arg), host.ctypes.data, hb.value - 1, ct.c_void_p(256), db.value,
                          None, ct.byref(h))
    assert rc == B.ENOMEM
    # stage sizes beyond the block kernel (more than 256 rows per stage block,
    # more than 64 inputs, or more than 64 general rows): the wide-stage
    # kernel, FP64 without refinement only; LDS bounds what it takes
    for nx, nu, ng in ((250, 10, 0), (80, 70, 0), (40, 8, 70)):
        big = B.Dims(2, [nx] * 3, [nu, nu, 0], [0, 0, 0], [0, 0, 0], [ng, ng, 0])
        arr1 = (ct.c_void_p * 1)(big.h)
        assert L.oqp_batch_bytes(arr1, 1, ct.byref(arg), ct.byref(hb), ct.byref(db)) == B.OK, (nx, nu, ng)
        for other in (B.default_arg(B.MODE_MIXED), B.default_arg(B.MODE_ROBUST), B.default_arg(ir_max=2)):
            rc = L.oqp_batch_bytes(arr1, 1, ct.byref(other), ct.byref(hb), ct.byref(db))
            assert rc == B.EINVAL and b"FP64 mode without refinement" in L.oqp_last_error(), (nx, nu, ng)
    huge = B.Dims(1, [4000] * 2, [8, 0], [0, 0], [0, 0], [0, 0])
    arr1 = (ct.c_void_p * 1)(huge.h)
    assert L.oqp_batch_bytes(arr1, 1, ct.byref(arg), ct.byref(hb), ct.byref(db)) == B.EINVAL
    # a large stage block is accepted (global-memory mode of the block kernel)
    ok = B.Dims(2, [128] * 3, [32, 32, 0], [0, 0, 0], [0, 0, 0], [32, 32, 0])
    arr1 = (ct.c_void_p * 1)(ok.h)
    assert L.oqp_batch_bytes(arr1, 1, ct.byref(arg), ct.byref(hb), ct.byref(db)) == B.OK
    # bad arguments
    bad = B.default_arg(gamma=1.5)
    assert L.oqp_batch_bytes(arr, 3, ct.byref(bad), ct.byref(hb), ct.byref(db)) == B.EINVAL
    bad = B.default_arg(warm_start=3)
    assert L.oqp_batch_bytes(arr, 3, ct.byref(bad), ct.byref(hb), ct.byref(db)) == B.EINVAL
    bad = B.default_arg(warm_start=2, cond_N=2)  # warm start does not combine with condensing
    assert L.oqp_batch_bytes(arr, 3, ct.byref(bad), ct.byref(hb), ct.byref(db)) == B.EINVAL
    ok = B.default_arg(warm_start=2)
    assert L.oqp_batch_bytes(arr, 3, ct.byref(ok), ct.byref(hb), ct.byref(db)) == B.OK
    # robust and balance modes: the array algorithm is built for the one-wave
    # variants and the block kernel, so they take the same kernels
    rob = B.default_arg(B.MODE_ROBUST)
    assert L.oqp_batch_bytes(arr, 3, ct.byref(rob), ct.byref(hb), ct.byref(db)) == B.OK
    big = B.Dims(2, [40] * 3, [8, 8, 0], [0, 0, 0], [0, 0, 0], [0, 0, 0])
    arr1 = (ct.c_void_p * 1)(big.h)
    hb0, db0 = ct.c_size_t(0), ct.c_size_t(0)
    assert L.oqp_batch_bytes(arr1, 1, ct.byref(B.default_arg()), ct.byref(hb0), ct.byref(db0)) == B.OK
    assert L.oqp_batch_bytes(arr1, 1, ct.byref(rob), ct.byref(hb), ct.byref(db)) == B.OK
    assert (hb.value, db.value) == (hb0.value, db0.value)
    bal = B.default_arg(B.MODE_BALANCE)
    assert bal.mode == B.MODE_BALANCE and bal.ir_max == 2 and rob.ir_max == 4
    assert L.oqp_batch_bytes(arr, 3, ct.byref(bal), ct.byref(hb), ct.byref(db)) == B.OK
    assert L.oqp_batch_bytes(arr1, 1, ct.byref(bal), ct.byref(hb), ct.byref(db)) == B.OK
    # refinement in the FP64 mode is not combined with slacks
    soft = B.Dims(2, [4] * 3, [2, 2, 0], [2, 2, 0], [0, 4, 4], [0, 0, 0], ns=[0, 2, 2])
    arr2 = (ct.c_void_p * 1)(soft.h)
    assert L.oqp_batch_bytes(arr2, 1, ct.byref(B.default_arg()), ct.byref(hb), ct.byref(db)) == B.OK
    assert L.oqp_batch_bytes(arr2, 1, ct.byref(B.default_arg(ir_max=2)), ct.byref(hb), ct.byref(db)) == B.EINVAL
    unknown = B.default_arg()
    unknown.mode = 5
    assert L.oqp_batch_bytes(arr, 3, ct.byref(unknown), ct.byref(hb), ct.byref(db)) == B.EINVAL
    assert L.oqp_batch_bytes(arr, 0, ct.byref(arg), ct.byref(hb), ct.byref(db)) == B.EINVAL


def test_bucket_choice_covers_instance():
    qp = W.mass_spring_chain8(0)
    L = B.lib()
    # smallest variant covering nx=16, nu=7, ng=0 is (16, 8, 0)
    cover = [(a, b, c) for a, b, c in B.variants() if a >= 16 and b >= 7]
    assert (16, 8, 0) in cover


def test_sol_object_host_errors():
    L = B.lib()
    qp = W.random_tiny(np.random.default_rng(3), 3, ng_max=2)
    d = B.Dims.of(qp)
    assert L.oqp_sol_bytes(None) == 0
    nb = L.oqp_sol_bytes(d.h)
    mem = B._aligned(nb, 64)
    h = ct.c_void_p()
    assert L.oqp_sol_init(d.h, mem.ctypes.data, nb - 8, ct.byref(h)) == B.ENOMEM
    assert L.oqp_sol_init(d.h, mem.ctypes.data + 8, nb, ct.byref(h)) == B.EINVAL
    assert L.oqp_sol_init(d.h, mem.ctypes.data, nb, ct.byref(h)) == B.OK
    out = np.zeros(16)
    assert L.oqp_sol_get_x(h, 0, B._p(out)) == B.ESTATE  # not filled yet
    assert L.oqp_sol_get_x(h, qp.N + 1, B._p(out)) == B.EINVAL
    st = B.Stat()
    assert L.oqp_sol_get_stat(h, ct.byref(st)) == B.ESTATE
