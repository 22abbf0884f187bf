"""The batch entry point that allocates nothing (oqp_batch_init_static):
its device records live in the library's static device region.  Results
must be bitwise those of the same batch in a caller-provided device buffer
(the same kernels run on the same records), on two batches in a row, the
second smaller than the first (it reuses the region the first one left);
a batch larger than the region is refused with OQP_ENOMEM."""
import ctypes as ct
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2003_02547_amd import binding as B  # noqa: E402
from paper_2003_02547_amd import workloads as W  # noqa: E402

KEYS = ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    B.lib()


def _same(a, b, what):
    ra, rb = a.results(), b.results()
    for i, (x, y) in enumerate(zip(ra, rb)):
        assert x.status == y.status and x.iters == y.iters, (what, i, x.status, y.status, x.iters, y.iters)
        assert np.array_equal(x.res, y.res), (what, i)
        for k in KEYS:
            assert np.array_equal(x.sol[k], y.sol[k]), (what, i, k)


def test_static_region_matches_caller_buffer_twice():
    first = [W.mass_spring_chain8(i) for i in range(96)] + [W.random_uneven(i) for i in range(8)]
    second = [W.mass_spring_chain4(s) for s in range(1, 9)] + [W.random_uneven(100 + i) for i in range(3)]
    for name, qps, mode in (("first", first, B.MODE_F64), ("second, smaller", second, B.MODE_MIXED)):
        say(f"static region: {name} batch ({len(qps)} instances, mode {mode})")
        arg = B.default_arg(mode)
        st = B.Batch(qps, arg, static=True)
        assert st.dev_ptr is None and st.dev_bytes <= 128 << 20
        st.load().solve().fetch().sync()
        ref = B.Batch(qps, arg).load().solve().fetch().sync()
        _same(st, ref, name)
        assert sum(r.status == B.SUCCESS for r in st.results()) >= len(qps) - 1
        del st, ref


def test_static_region_refuses_a_batch_too_large():
    qps = [W.mass_spring_chain8(i) for i in range(320)]  # ~0.6 MB of records each
    say("static region: a batch above its size")
    dims = [B.Dims.of(q) for q in qps]
    arr = (ct.c_void_p * len(dims))(*[d.h for d in dims])
    arg = B.default_arg()
    hb, db = ct.c_size_t(0), ct.c_size_t(0)
    L = B.lib()
    assert L.oqp_batch_bytes(arr, len(dims), ct.byref(arg), ct.byref(hb), ct.byref(db)) == 0
    assert db.value > (128 << 20)
    host = np.zeros(hb.value + 64, dtype=np.uint8)
    base = host.ctypes.data + ((-host.ctypes.data) % 64)
    h = ct.c_void_p()
    rc = L.oqp_batch_init_static(arr, len(dims), ct.byref(arg), base, hb.value, None, ct.byref(h))
    assert rc == -2, rc  # OQP_ENOMEM
    msg = L.oqp_last_error().decode()
    assert "static region" in msg and str(db.value) in msg, msg
