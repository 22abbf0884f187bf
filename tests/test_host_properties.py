"""Property checks of the host side of the C-ABI (no GPU): for random stage
sizes and data, the QP getters return what the setters stored, condensed
stage sizes keep every constraint and input of the QP (Section 3.5), and the
batch sizes grow with the batch."""
import ctypes as ct

import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

from paper_2003_02547_amd import binding as B  # noqa: E402
from paper_2003_02547_amd import workloads as W  # noqa: E402

FIELDS = ("A", "B", "b", "Q", "S", "R", "q", "r", "idxbu", "lbu", "ubu", "idxbx", "lbx", "ubx", "D", "C", "lg", "ug")


def tiny_from(seed, N):
    rng = np.random.default_rng(seed)
    return W.random_tiny(rng, N, nx_range=(0, 5), nu_range=(0, 4), nb_frac=0.5, ng_max=3, x0_mode="free")


@settings(max_examples=40, deadline=None)
@given(seed=st.integers(0, 10 ** 6), N=st.integers(1, 8))
def test_getters_return_what_setters_stored(seed, N):
    qp = tiny_from(seed, N)
    q = B.Qp(qp)
    back = B.qp_fields(q.h, q.dims)
    for f in FIELDS:
        for n, (a, b) in enumerate(zip(getattr(back, f), getattr(qp, f))):
            a, b = np.asarray(a), np.asarray(b)
            assert a.shape == b.shape and np.array_equal(a, b), (f, n)


@settings(max_examples=60, deadline=None)
@given(seed=st.integers(0, 10 ** 6), N=st.integers(1, 12), cond_N=st.integers(1, 15))
def test_condensed_sizes_keep_the_qp(seed, N, cond_N):
    qp = tiny_from(seed, N)
    d = B.Dims.condensed(qp, cond_N).sizes()
    N2 = min(cond_N, N)
    assert len(d["nx"]) == N2 + 1
    nbu, nbx, ng = qp.nbu, qp.nbx, qp.ng
    # every input and input box survives, once
    assert sum(d["nu"]) == sum(qp.nu) and sum(d["nbu"]) == sum(nbu)
    # every constraint row survives: interior state boxes become general rows
    assert sum(d["nbu"]) + sum(d["nbx"]) + sum(d["ng"]) == sum(nbu) + sum(nbx) + sum(ng)
    # block-start states, the terminal stage as it is
    assert d["nx"][0] == qp.nx[0] and d["nx"][-1] == qp.nx[N] and d["nu"][-1] == qp.nu[N]
    assert d["ng"][-1] == ng[N] and d["nbx"][-1] == nbx[N]
    # near-equal blocks
    q, r = divmod(N, N2)
    starts = [b * q + min(b, r) for b in range(N2)]
    assert [qp.nx[s] for s in starts] == d["nx"][:-1]


@settings(max_examples=20, deadline=None)
@given(seed=st.integers(0, 10 ** 6), count=st.integers(1, 6))
def test_batch_sizes_grow_with_the_batch(seed, count):
    L = B.lib()
    qps = [tiny_from(seed + k, 1 + (seed + k) % 6) for k in range(count + 1)]
    dims = [B.Dims.of(q) for q in qps]
    arg = B.default_arg()
    sizes = []
    for c in (count, count + 1):
        arr = (ct.c_void_p * c)(*[d.h for d in dims[:c]])
        hb, db = ct.c_size_t(), ct.c_size_t()
        assert L.oqp_batch_bytes(arr, c, ct.byref(arg), ct.byref(hb), ct.byref(db)) == B.OK
        sizes.append((hb.value, db.value))
    assert sizes[1][0] > sizes[0][0] and sizes[1][1] > sizes[0][1]
