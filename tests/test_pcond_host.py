"""Host-side checks of partial condensing at the C-ABI (no GPU needed): the
condensed stage sizes equal those of the oracle's condensed QP (Section 3.5),
the QP getters return what the setters stored, and batch planning accepts or
rejects condensing before any device call."""
import ctypes as ct

import numpy as np
import pytest

from oracle import pcond as PC
from paper_2003_02547_amd import binding as B
from paper_2003_02547_amd import workloads as W


def _cases():
    rng = np.random.default_rng(9)
    return [
        ("chain8", W.mass_spring_chain8(0), [5, 10, 15, 30, 31, 100]),
        ("chain4", W.mass_spring_chain4(1), [1, 2, 3, 4, 10]),
        ("uneven", W.random_uneven(2), [3, 7]),
        ("tiny", W.random_tiny(rng, 7, nx_range=(1, 4), nu_range=(0, 3), ng_max=2), [1, 2, 3, 6, 7]),
    ]


@pytest.mark.parametrize("name,qp,n2s", _cases(), ids=[c[0] for c in _cases()])
def test_condensed_dims_match_oracle(name, qp, n2s):
    for N2 in n2s:
        d = B.Dims.condensed(qp, N2).sizes()
        cq = PC.condense(qp, N2)
        assert d["nx"] == list(cq.nx) and d["nu"] == list(cq.nu), (name, N2)
        assert d["nbu"] == [len(i) for i in cq.idxbu], (name, N2)
        assert d["nbx"] == [len(i) for i in cq.idxbx], (name, N2)
        assert d["ng"] == [np.asarray(g).shape[0] for g in cq.D], (name, N2)


def test_qp_getters_return_what_the_setters_stored():
    qp = W.random_tiny(np.random.default_rng(4), 4, nx_range=(1, 4), nu_range=(0, 3), ng_max=2)
    q = B.Qp(qp)
    back = B.qp_fields(q.h, q.dims)
    for f in ("A", "B", "b", "Q", "S", "R", "q", "r", "idxbu", "lbu", "ubu", "idxbx", "lbx", "ubx", "D", "C", "lg",
              "ug"):
        for n, (a, b) in enumerate(zip(getattr(back, f), getattr(qp, f))):
            assert np.array_equal(np.asarray(a), np.asarray(b)), (f, n)


def test_condensing_batch_plan():
    L = B.lib()
    qps = [W.mass_spring_chain8(i) for i in range(2)]
    dims = [B.Dims.of(q) for q in qps]
    arr = (ct.c_void_p * 2)(*[d.h for d in dims])
    hb, db = ct.c_size_t(), ct.c_size_t()
    plain = B.default_arg()
    assert L.oqp_batch_bytes(arr, 2, ct.byref(plain), ct.byref(hb), ct.byref(db)) == B.OK
    h0, d0 = hb.value, db.value
    cond = B.default_arg(cond_N=5)
    assert L.oqp_batch_bytes(arr, 2, ct.byref(cond), ct.byref(hb), ct.byref(db)) == B.OK
    assert db.value != d0 and hb.value != h0
    # negative horizon
    assert L.oqp_batch_bytes(arr, 2, ct.byref(B.default_arg(cond_N=-1)), ct.byref(hb), ct.byref(db)) == B.EINVAL
    # full condensing (one block of 30 stages: 210 inputs, 232 general rows):
    # the wide-stage kernel, FP64 only
    assert L.oqp_batch_bytes(arr, 2, ct.byref(B.default_arg(cond_N=1)), ct.byref(hb), ct.byref(db)) == B.OK
    rc = L.oqp_batch_bytes(arr, 2, ct.byref(B.default_arg(B.MODE_MIXED, cond_N=1)), ct.byref(hb), ct.byref(db))
    assert rc == B.EINVAL and b"condensed" in L.oqp_last_error()
    # the server does not condense
    cfg = B.ServerCfg()
    L.oqp_server_cfg_default(ct.byref(cfg))
    h = ct.c_void_p()
    rc = L.oqp_server_init(ct.byref(cfg), ct.byref(cond), None, 0, None, 0, None, 0, ct.byref(h))
    assert rc == B.EINVAL and b"condensing" in L.oqp_last_error()


def test_condensed_dims_errors():
    L = B.lib()
    d = B.Dims.of(W.mass_spring_chain4(1))
    assert L.oqp_pcond_dims_bytes(d.h, 0) == 0
    assert L.oqp_pcond_dims_bytes(d.h, 3) == L.oqp_dims_bytes(3)
    assert L.oqp_pcond_dims_bytes(d.h, 50) == L.oqp_dims_bytes(10)  # clipped to N
    mem = B._aligned(L.oqp_dims_bytes(3))
    h = ct.c_void_p()
    assert L.oqp_pcond_dims(d.h, 0, mem.ctypes.data, mem.nbytes, ct.byref(h)) == B.EINVAL
    assert L.oqp_pcond_dims(d.h, 3, mem.ctypes.data, 8, ct.byref(h)) == B.ENOMEM
    assert L.oqp_pcond_dims(d.h, 3, mem.ctypes.data, mem.nbytes, ct.byref(h)) == B.OK
