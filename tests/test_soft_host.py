"""Host side of soft constraints in the C-ABI (no GPU): slack counts in the
dims, the soft setters and getters with their validation, the batch sizing
rules of a batch with slacks (FP64 mode, no condensing, warm starts allowed; the
soft records larger than the hard ones) and packed requests with slacks."""
import ctypes as ct

import numpy as np
import pytest

from paper_2003_02547_amd import binding as B
from paper_2003_02547_amd import workloads as W

_P = ct.POINTER(ct.c_double)
_PI = ct.POINTER(ct.c_int)


def soft_qp(seed=3, N=4):
    rng = np.random.default_rng(seed)
    qp = W.random_tiny(rng, N, nx_range=(2, 5), nu_range=(1, 3), ng_max=2)
    return W.soften_random(qp, rng)


def test_dims_slack_count_is_checked():
    L = B.lib()
    d = B.Dims(2, [2, 2, 2], [1, 1, 0], [1, 1, 0], [2, 2, 2], [0, 1, 0])
    assert L.oqp_dims_set_soft(d.h, 1, 4) == B.OK           # nbu + nbx + ng = 4
    assert L.oqp_dims_set_soft(d.h, 1, 5) == B.EINVAL
    assert L.oqp_dims_set_soft(d.h, 3, 0) == B.EINVAL        # stage out of range
    assert L.oqp_dims_set_soft(d.h, 0, -1) == B.EINVAL
    # stage sizes shrunk after the slacks were set: caught when a QP is made
    assert L.oqp_dims_set_stage(d.h, 1, 2, 1, 0, 1, 0) == B.OK
    mem = np.zeros(L.oqp_qp_bytes(d.h) + 64, dtype=np.uint8)
    base = mem.ctypes.data + ((-mem.ctypes.data) % 16)
    h = ct.c_void_p()
    assert L.oqp_qp_init(d.h, base, mem.nbytes - 64, ct.byref(h)) == B.EINVAL


def test_soft_setters_round_trip_and_validate():
    qp = soft_qp()
    q = B.Qp(qp)
    back = B.qp_fields(q.h, q.dims)
    for k in ("idxs",) + B.SOFT_FIELDS:
        for n in range(qp.N + 1):
            assert np.array_equal(np.asarray(getattr(back, k)[n]), np.asarray(getattr(qp, k)[n])), (k, n)
    L = B.lib()
    n = next(i for i in range(qp.N + 1) if len(qp.idxs[i]) >= 2)
    ns = len(qp.idxs[n])
    nc = qp.nbu[n] + qp.nbx[n] + qp.ng[n]
    ones = np.ones(ns)

    def call(idx, Z=ones, z=ones):
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        return L.oqp_qp_set_soft(q.h, n, idx.ctypes.data_as(_PI), *[a.ctypes.data_as(_P) for a in (Z, Z, z, z, ones,
                                                                                                      ones)])

    assert call(qp.idxs[n]) == B.OK
    rep = np.array(qp.idxs[n]); rep[1] = rep[0]
    assert call(rep) == B.EINVAL                                     # a row twice
    out = np.array(qp.idxs[n]); out[0] = nc
    assert call(out) == B.EINVAL                                     # row out of range
    assert call(qp.idxs[n], Z=-ones) == B.EINVAL                     # negative Hessian
    assert call(qp.idxs[n], z=np.full(ns, np.inf)) == B.EINVAL       # not finite


def _bytes(qps, arg):
    L = B.lib()
    dims = [B.Dims.of(q) for q in qps]
    arr = (ct.c_void_p * len(dims))(*[d.h for d in dims])
    hb, db = ct.c_size_t(), ct.c_size_t()
    rc = L.oqp_batch_bytes(arr, len(dims), ct.byref(arg), ct.byref(hb), ct.byref(db))
    return rc, hb.value, db.value


def test_soft_batch_sizing_rules():
    hard = W.mass_spring_chain8(0)
    soft = W.mass_spring_chain8_soft(0)
    rc, _, dh = _bytes([hard], B.default_arg())
    assert rc == B.OK
    rc, _, ds = _bytes([soft], B.default_arg())
    assert rc == B.OK and ds > dh                  # slack blocks in every record
    for arg in (B.default_arg(B.MODE_MIXED), B.default_arg(B.MODE_ABS), B.default_arg(B.MODE_ROBUST),
                B.default_arg(B.MODE_BALANCE), B.default_arg(cond_N=5)):
        assert _bytes([soft], arg)[0] == B.EINVAL
        assert _bytes([hard, soft], arg)[0] == B.EINVAL   # one soft instance makes the batch soft
    assert _bytes([soft], B.default_arg(warm_start=2))[0] == B.OK   # warm starts take slack guesses
    # a hard QP in a soft batch takes the soft records too
    rc, _, dm = _bytes([hard, soft], B.default_arg())
    assert rc == B.OK and dm >= 2 * ds - 4096


def test_packed_requests_with_slacks():
    """A packed request with slacks takes the soft layout (a larger
    footprint) and a kernel group of its own, offset by the number of
    groups; without slacks it is what it was."""
    L = B.lib()
    hard, soft = B.Packed(W.mass_spring_chain8(1)), B.Packed(W.mass_spring_chain8_soft(1))
    ngroups = L.oqp_variant_count() + 7  # one-wave variants, six block builds, the wide-stage kernel
    assert hard.variant < ngroups and soft.variant == hard.variant + ngroups
    assert soft.footprint > hard.footprint and soft.nbytes > hard.nbytes
    none = B.Packed(W.soften(W.mass_spring_chain8(1), lambda n, q: [], 1.0, 1.0, 1.0, 1.0))
    assert none.variant == hard.variant and none.footprint == hard.footprint


def test_soft_workloads():
    qp = W.mass_spring_chain8_soft(5)
    assert qp.ns[0] == 0 and all(qp.ns[n] == qp.nbx[n] for n in range(1, qp.N + 1))
    # first x0 draw kept: equal to the hard workload wherever no redraw was needed
    for i in range(12):
        h, s = W.random_uneven(i), W.random_uneven_soft(i)
        assert (h.meta["redraws"] == 0) == np.array_equal(h.lbx[0], s.lbx[0]), i
