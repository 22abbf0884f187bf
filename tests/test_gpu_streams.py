"""Concurrent kernel groups on extra streams: the solve forks from the batch
stream and joins back, and every instance's result is bit for bit the one of
the single-stream solve (instances are independent of where their group
runs), FP64 and mixed (whose FP64 fallback runs on its group's stream)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2003_02547_amd import binding as B  # noqa: E402
from paper_2003_02547_amd import workloads as W  # noqa: E402

KEYS = ("u", "x", "pi", "lam_l", "lam_u", "t_l", "t_u")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    B.lib()


@pytest.mark.parametrize("mode,given", [(B.MODE_F64, False), (B.MODE_MIXED, False), (B.MODE_F64, True)])
def test_extra_streams_bitwise_equal(mode, given):
    qps = [W.random_uneven(i) for i in range(24)] + [W.mass_spring_chain4(s) for s in range(4)]
    print(f"extra streams vs one stream, mode {mode}, caller's streams {given}", flush=True)
    sys.stdout.flush()
    one = B.Batch(qps, B.default_arg(mode)).load().solve().fetch().sync().results()
    extra = [torch.cuda.Stream() for _ in range(3)] if given else 3
    many = B.Batch(qps, B.default_arg(mode), streams=extra)
    groups = {many.variant(i)[0] for i in range(len(qps))}
    assert len(groups) >= 4
    res = many.load().solve().fetch().sync().results()
    # a second solve reuses the fork/join events
    res2 = many.solve().fetch().sync().results()
    for i, (a, b, c) in enumerate(zip(one, res, res2)):
        assert a.status == b.status == c.status and a.iters == b.iters == c.iters, i
        for k in KEYS:
            assert np.array_equal(a.sol[k], b.sol[k]) and np.array_equal(a.sol[k], c.sol[k]), (i, k)
    assert B.lib().oqp_batch_release(many.h) == 0


def test_batches_in_flight_bitwise_equal():
    """Three copies of a batch, each on its own stream, solved back to back
    without waiting in between (the benchmark's batches in flight): every copy
    returns bitwise the result of the batch solved alone, twice over."""
    qps = [W.mass_spring_chain8(i) for i in range(64)] + [W.random_uneven(i) for i in range(16)]
    print("three batches in flight vs one batch alone", flush=True)
    sys.stdout.flush()
    alone = B.Batch(qps).load().solve().fetch().sync().results()
    copies = [B.Batch(qps, stream=torch.cuda.Stream()) for _ in range(3)]
    for c in copies:
        c.load()
    for _ in range(2):
        for c in copies:
            c.solve()
    torch.cuda.synchronize()
    for c in copies:
        res = c.fetch().sync().results()
        for i, (a, r) in enumerate(zip(alone, res)):
            assert a.status == r.status and a.iters == r.iters, i
            for k in KEYS:
                assert np.array_equal(a.sol[k], r.sol[k], equal_nan=True), (i, k)
