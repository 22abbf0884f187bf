"""Oracle solves of many instances on the host cores, for the parity tests
that compare whole batches (the C oracle releases the interpreter lock while
it runs, so threads run it in parallel)."""
import concurrent.futures as cf
import os

from oracle import oracle as O


def solve_many(qps, idx, arg=None):
    """{i: oracle result of qps[i]} for i in idx."""
    idx = list(idx)
    threads = max(1, min(16, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(threads) as ex:
        return dict(zip(idx, ex.map(lambda i: O.solve(qps[i], arg), idx)))


def kkt_many(qps, sols, idx):
    """{i: host KKT residual of sols[i]} for i in idx (the oracle's residual
    routine in FP64)."""
    idx = list(idx)
    threads = max(1, min(16, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(threads) as ex:
        return dict(zip(idx, ex.map(lambda i: O.kkt_res(qps[i], sols[i]), idx)))
