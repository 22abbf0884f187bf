"""Continuous-batching server on the GPU.

The bar: a request served in a mix (admitted while other requests of other
sizes are running, launched in groups with whatever else is queued) returns
exactly the result it gets when solved alone in a batch of one: same status,
iteration count and bitwise-equal solution (the kernel of a variant computes
each instance independently of its neighbours).  The lone results are tied
to the oracle by the batch parity tests; here they are also checked against
the oracle's status and the host-evaluated KKT residual.
"""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
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


def mixed_pool():
    qps = [W.random_uneven(i) for i in range(10)]
    qps += [W.mass_spring_chain4(s) for s in range(1, 5)]
    qps += [W.mass_spring_chain8(i) for i in range(4)]
    rng = np.random.default_rng(11)
    qps += [W.random_tiny(rng, int(rng.integers(1, 6)), ng_max=2) for _ in range(6)]
    return qps


def serve_all(server, packed, order, spacing_s=0.0):
    """Submit in the given order, driving progress between submissions so
    later requests are admitted while earlier ones run; wait for all."""
    tickets = {}
    pending = list(order)
    deadline = time.time() + 60
    while pending or any(server.poll(t) is None for t in tickets.values()):
        assert time.time() < deadline, "server made no progress"
        if pending:
            t = server.submit(packed[pending[0]])
            if t is not None:
                tickets[pending.pop(0)] = t
        server.progress()
        if spacing_s:
            time.sleep(spacing_s)
    return tickets


def check_same_as_alone(server, qps, tickets, arg):
    for i, t in tickets.items():
        st = server.poll(t)
        got = server.solution(t)
        alone = B.solve([qps[i]], arg)[0]
        assert st.status == alone.status and st.iters == alone.iters, (i, st.status, alone.status)
        for k in KEYS:
            assert np.array_equal(got[k], alone.sol[k]), (i, k)


@pytest.mark.parametrize("mode", [B.MODE_F64, B.MODE_MIXED])
def test_served_in_mix_equals_alone(mode):
    qps = mixed_pool()
    arg = B.default_arg(mode)
    packed = [B.Packed(q, pinned=True) for q in qps]
    say(f"serve mix: {len(qps)} requests, mode {mode}")
    srv = B.Server(arg, dev_bytes=512 << 20, nstreams=4, max_launch=8)
    try:
        order = list(np.random.default_rng(5).permutation(len(qps)))
        tickets = serve_all(srv, packed, order, spacing_s=0.0005)
        s = srv.stats()
        assert s["completed"] == len(qps) and s["launches"] >= 2
        check_same_as_alone(srv, qps, tickets, arg)
        tol = 1e-8 if mode == B.MODE_F64 else 1e-6
        for i, t in tickets.items():
            st = srv.poll(t)
            if st.status == B.SUCCESS:
                assert O.kkt_res(qps[i], srv.solution(t)) <= tol + 1e-12, i
            elif mode == B.MODE_F64 and i >= 10:  # the small ones are cheap for the oracle
                assert O.solve(qps[i], O.Arg.with_tol(tol)).status != O.SUCCESS, i
        for t in tickets.values():
            srv.release(t)
        assert srv.stats()["dev_used"] == 0
    finally:
        srv.close()


def test_admission_by_device_footprint():
    """An arena that holds only a few requests refuses the rest with
    OQP_EBUSY and admits them once finished requests are released."""
    qps = [W.mass_spring_chain8(i) for i in range(12)]
    packed = [B.Packed(q, pinned=True) for q in qps]
    fp = packed[0].footprint
    say(f"admission: footprint {fp} bytes, arena for 3")
    srv = B.Server(B.default_arg(), dev_bytes=3 * fp + fp // 2, nstreams=3)
    try:
        t = [srv.submit(p) for p in packed[:4]]
        assert all(x is not None for x in t[:3]) and t[3] is None
        s = srv.stats()
        assert s["dev_used"] == 3 * fp and s["rejected"] == 1 and s["dev_used"] <= s["dev_arena"]
        done = {}
        nxt = 3
        live = list(zip(range(3), t[:3]))
        deadline = time.time() + 60
        while live:
            assert time.time() < deadline
            srv.progress()
            for i, tk in list(live):
                if srv.poll(tk) is not None:
                    done[i] = (srv.poll(tk).status, srv.solution(tk)["u"].copy())
                    srv.release(tk)
                    live.remove((i, tk))
                    if nxt < len(packed):
                        tk2 = srv.submit(packed[nxt])
                        assert tk2 is not None
                        live.append((nxt, tk2))
                        nxt += 1
        assert len(done) == len(qps)
        s = srv.stats()
        assert s["dev_peak"] <= 3 * fp and s["dev_used"] == 0 and s["completed"] == len(qps)
        ref = B.solve(qps, B.default_arg())
        for i in range(len(qps)):
            assert done[i][0] == ref[i].status
            assert np.array_equal(done[i][1], ref[i].sol["u"])
    finally:
        srv.close()


def test_replay_poisson_matches_batch():
    """Native replay of a Poisson schedule over a pool of uneven instances:
    every request finishes with the status and iteration count of the batch
    solve of the same instance, and latencies are positive."""
    pool = [W.random_uneven(i) for i in range(24)]
    packed = [B.Packed(q, pinned=True) for q in pool]
    times, idx = W.serving_stream(2000.0, 0.1, len(pool), seed=1)
    say(f"replay: {len(times)} arrivals over 0.1 s")
    srv = B.Server(B.default_arg(), dev_bytes=2 << 30, nstreams=8)
    try:
        lat, stats, wall = srv.replay([packed[i] for i in idx], times, timeout=60.0)
        assert wall >= times[-1]
        assert np.all(lat > 0)
        ref = B.solve(pool, B.default_arg())
        for k, i in enumerate(idx):
            assert stats[k].status == ref[i].status and stats[k].iters == ref[i].iters, (k, i)
        s = srv.stats()
        assert s["completed"] == len(times) and s["dev_used"] == 0
    finally:
        srv.close()


def test_server_errors():
    srv = B.Server(B.default_arg(), dev_bytes=1 << 18, nstreams=2)
    try:
        big = B.Packed(W.mass_spring_chain8(0), pinned=True)
        assert big.footprint > (1 << 18)
        with pytest.raises(B.OqpError) as e:
            srv.submit(big)
        assert e.value.code == B.ENOMEM
        small = B.Packed(W.random_tiny(np.random.default_rng(1), 2), pinned=True)
        t = srv.submit(small)
        assert t is not None
        with pytest.raises(B.OqpError) as e:
            srv.release(t)  # not finished yet
        assert e.value.code == B.ESTATE
        deadline = time.time() + 30
        while srv.poll(t) is None:
            assert time.time() < deadline
            srv.progress()
        srv.release(t)
        with pytest.raises(B.OqpError):
            srv.poll(t)  # stale ticket
    finally:
        srv.close()


def test_soft_requests_served_in_mix_equal_alone():
    """Requests with slacks (soft constraints, Section 2.2) take a kernel
    group of their own and the soft builds; served among requests without
    slacks, each equals its solve alone in a batch of one, slack blocks
    included, and reaches the oracle's KKT tolerance."""
    qps = [W.random_uneven_soft(i) for i in range(8)] + [W.mass_spring_chain8_soft(i) for i in (0, 222)]
    qps += mixed_pool()[10:18]
    nsoft = 10
    arg = B.default_arg()
    packed = [B.Packed(q, pinned=True) for q in qps]
    say(f"serve mix with slacks: {len(qps)} requests, {nsoft} with slacks")
    srv = B.Server(arg, dev_bytes=512 << 20, nstreams=4, max_launch=8)
    try:
        order = list(np.random.default_rng(9).permutation(len(qps)))
        tickets = serve_all(srv, packed, order, spacing_s=0.0005)
        assert srv.stats()["completed"] == len(qps)
        for i, t in tickets.items():
            st = srv.poll(t)
            got = srv.solution(t)
            alone = B.solve([qps[i]], arg)[0]
            assert st.status == alone.status and st.iters == alone.iters, (i, st.status, alone.status)
            for k in alone.sol:
                assert np.array_equal(got[k], alone.sol[k]), (i, k)
            if i < nsoft:
                assert st.status == B.SUCCESS and "s_l" in got, i
                assert O.kkt_res(qps[i], got) <= 1e-8 * 1.01, i
        for t in tickets.values():
            srv.release(t)
    finally:
        srv.close()
    # requests with slacks need a server in the FP64 mode
    mixed = B.Server(B.default_arg(B.MODE_MIXED), dev_bytes=64 << 20, nstreams=2)
    try:
        with pytest.raises(B.OqpError):
            mixed.submit(packed[0])
    finally:
        mixed.close()


@pytest.mark.parametrize("block", [1, 3])
def test_iteration_blocks_equal_alone(block):
    """Iteration blocks: each launch runs at most `block` IPM iterations and
    the unfinished requests are launched again (with the ones that arrived
    meanwhile) from their device-resident iterates.  Statuses, iteration
    counts (summed over the launches) and solutions are bitwise those of the
    request solved alone in one launch; requests that stop at the iteration
    limit stop there too."""
    qps = mixed_pool()
    arg = B.default_arg(B.MODE_F64)
    packed = [B.Packed(q, pinned=True) for q in qps]
    say(f"serve with iteration blocks of {block}: {len(qps)} requests")
    srv = B.Server(arg, dev_bytes=512 << 20, nstreams=4, max_launch=8, iter_block=block)
    try:
        order = list(np.random.default_rng(7).permutation(len(qps)))
        tickets = serve_all(srv, packed, order, spacing_s=0.0005)
        s = srv.stats()
        assert s["completed"] == len(qps)
        # more launches than a whole-solve server needs: requests come back
        assert s["launches"] >= max(r.iters for r in B.solve(qps, arg)) // block
        check_same_as_alone(srv, qps, tickets, arg)
        for t in tickets.values():
            srv.release(t)
    finally:
        srv.close()
    # the iteration limit is kept across launches
    lim = B.default_arg(B.MODE_F64, iter_max=5)
    srv = B.Server(lim, dev_bytes=256 << 20, nstreams=3, max_launch=8, iter_block=block)
    try:
        tickets = serve_all(srv, packed[:8], list(range(8)))
        check_same_as_alone(srv, qps[:8], tickets, lim)
        for i, t in tickets.items():
            assert srv.poll(t).iters <= 5
    finally:
        srv.close()


def test_iteration_blocks_need_fp64_mode():
    with pytest.raises(B.OqpError):
        B.Server(B.default_arg(B.MODE_MIXED), dev_bytes=64 << 20, nstreams=2, iter_block=2)
