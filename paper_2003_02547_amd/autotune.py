"""Autotuner for the kernel choice of the batched IPM.

An instance goes to a one-wave kernel variant when the variant's padded
stage block (nx + nu) is at most a bound, else to the 256-thread block kernel
(`oqp_set_wave_max`).  The tuner times both kernels on batches of random
stable OCP QPs of each variant's size, on the current device, and sets the
bound to the largest stage block up to which the one-wave kernel wins for
every variant.  Timing runs through the library (device events on the batch
stream); no solver arithmetic lives here.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import binding as B
from . import workloads as W


def choose_bound(timings: Dict[Tuple[int, int, int], Tuple[float, float]]) -> int:
    """Largest padded stage block nx + nu such that, for every variant with a
    block no larger, the one-wave time is below the block-kernel time.
    timings maps (nx, nu, ng) -> (one-wave seconds, block seconds)."""
    by_nz: Dict[int, List[bool]] = {}
    for (nx, nu, ng), (tw, tb) in timings.items():
        by_nz.setdefault(nx + nu, []).append(tw < tb)
    bound = 0
    for nz in sorted(by_nz):
        if not all(by_nz[nz]):
            break  # the bound is one threshold: stop at the first block size that loses
        bound = nz
    return bound


def _batch(nx: int, nu: int, ng: int, count: int, N: int, seed: int) -> List:
    rng = np.random.default_rng(np.random.SeedSequence([11, nx, nu, ng, seed]))
    base = W.random_stable(rng, nx, nu, N, ng=ng)
    return [base] * count


def _time(qps: Sequence, wave_max: int, reps: int) -> float:
    import torch
    old = B.set_wave_max(wave_max)
    try:
        b = B.Batch(qps, B.default_arg()).load()
        b.solve()
        torch.cuda.synchronize()
        st = b.stream
        best = float("inf")
        for _ in range(reps):
            s = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            s.record(st)
            b.solve()
            e.record(st)
            torch.cuda.synchronize()
            best = min(best, s.elapsed_time(e) * 1e-3)
        return best
    finally:
        B.set_wave_max(old)


def tune(count: int = 256, N: int = 30, reps: int = 2, apply: bool = True, seed: int = 0) -> dict:
    """Time every one-wave variant against the block kernel and (optionally)
    apply the resulting bound.  Returns {"bound": b, "timings": {...}}."""
    timings = {}
    for nx, nu, ng in B.variants():
        # the variant's own size (one input less when nu > 1, so the
        # instance is padded as real ones are)
        qps = _batch(nx, max(1, nu - 1) if nu > 1 else nu, ng, count, N, seed)
        tw = _time(qps, 64, reps)
        tb = _time(qps, 0, reps)
        timings[(nx, nu, ng)] = (tw, tb)
    bound = choose_bound(timings)
    if apply:
        B.set_wave_max(bound)
    return {"bound": bound, "timings": {f"{k[0]}x{k[1]}x{k[2]}": v for k, v in timings.items()}}


if __name__ == "__main__":
    import json

    print(json.dumps(tune(), indent=1))
