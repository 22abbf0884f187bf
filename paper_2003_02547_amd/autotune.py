"""Autotuners of the batched IPM's kernel choice and launch schedule.

An instance goes to a one-wave kernel variant when the variant's padded
stage block (nx + nu) is at most a bound and the variant is enabled, else to
the 256-thread block kernel (`oqp_set_wave_max`, `oqp_set_variant_mask`).

* `tune`: times both kernels on batches of random stable OCP QPs of each
  variant's size and sets the bound to the largest stage block up to which
  the one-wave kernel wins for every variant;
* `tune_schedule`: for a given batch, chooses the kernel family of each
  kernel group (one-wave variant or block kernel) from timings of the
  group's own instances, then the launch schedule of the groups (extra
  streams, LDS split of the block groups) from timings of the whole batch.

Timing runs through the library (device events on the batch stream); no
solver arithmetic lives here.
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



# ---------------------------------------------------------------------------
# Schedule of a given batch: kernel family per kernel group, then the launch
# schedule of the groups (concurrent streams, LDS split of the block groups)
# ---------------------------------------------------------------------------

def choose_variant_mask(timings: Dict[int, Tuple[float, float]], base_mask: int) -> int:
    """Keep bit v of base_mask when variant v's instances solve faster on the
    one-wave kernel than on the block kernel (timings: v -> (one-wave
    seconds, block seconds)); clear it otherwise."""
    mask = base_mask
    for v, (tw, tb) in timings.items():
        if not tw < tb:
            mask &= ~(1 << v)
    return mask


def choose_launch(timings: Dict[Tuple[int, int], float]) -> Tuple[int, int]:
    """(extra streams, LDS split) with the shortest time; a tie goes to fewer
    streams, then to the split (the defaults)."""
    if not timings:
        raise ValueError("no timings")
    return min(timings, key=lambda k: (timings[k], k[0], -k[1]))


def _time_batch(qps: Sequence, arg, reps: int, streams: int = 0) -> float:
    import torch
    b = B.Batch(qps, arg, streams=streams).load()
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


_schedules: Dict[tuple, dict] = {}


def batch_signature(qps: Sequence, arg=None) -> tuple:
    """Kernel groups of a batch under the current kernel choice, with their
    instance counts (the key the tuned schedules are kept under)."""
    b = B.Batch(qps, arg or B.default_arg())
    counts: Dict[int, int] = {}
    for i in range(len(qps)):
        g = b.variant(i)[0]
        counts[g] = counts.get(g, 0) + 1
    return tuple(sorted(counts.items()))


def tune_schedule(qps: Sequence, arg=None, reps: int = 2, stream_options: Sequence[int] = (0, 1, 3),
                  apply: bool = True, use_cache: bool = True) -> dict:
    """Tune the schedule of this batch on the current device:

    1. kernel family per kernel group: the instances of each one-wave variant
       present are timed on that variant and on the block kernel, and the
       variant stays enabled only where it wins (oqp_set_variant_mask);
    2. launch schedule: the whole batch with the chosen kernels, timed for
       every number of extra streams in stream_options, with and without the
       LDS split of the block groups (oqp_set_lds_split).

    Returns {"variant_mask", "streams", "lds_split", "family", "launch"}; with
    apply, the mask and the split are set process wide (the number of extra
    streams is a batch argument: pass it to Batch).  Schedules are cached by
    the batch's kernel-group signature."""
    arg = arg or B.default_arg()
    L = B.lib()
    sig = batch_signature(qps, arg) + ((arg.mode,),)
    if use_cache and sig in _schedules:
        out = _schedules[sig]
    else:
        base_mask = L.oqp_get_variant_mask()
        old_split = L.oqp_get_lds_split()
        nv = L.oqp_variant_count()
        b = B.Batch(qps, arg)
        groups: Dict[int, List[int]] = {}
        for i in range(len(qps)):
            g = b.variant(i)[0]
            if g < nv:
                groups.setdefault(g, []).append(i)
        del b
        family = {}
        try:
            for v, idx in sorted(groups.items()):
                sub = [qps[i] for i in idx]
                L.oqp_set_variant_mask(base_mask)
                tw = _time_batch(sub, arg, reps)
                L.oqp_set_variant_mask(base_mask & ~(1 << v))
                tb = _time_batch(sub, arg, reps)
                family[v] = (tw, tb)
            mask = choose_variant_mask(family, base_mask)
            L.oqp_set_variant_mask(mask)
            launch = {}
            for split in (1, 0):
                L.oqp_set_lds_split(split)
                for k in stream_options:
                    launch[(int(k), split)] = _time_batch(qps, arg, reps, streams=int(k))
            streams, split = choose_launch(launch)
        finally:
            L.oqp_set_variant_mask(base_mask)
            L.oqp_set_lds_split(old_split)
        out = {"variant_mask": int(mask), "streams": int(streams), "lds_split": int(split),
               "family": {int(v): t for v, t in family.items()},
               "launch": {f"{k[0]}x{k[1]}": t for k, t in launch.items()}}
        _schedules[sig] = out
    if apply:
        L.oqp_set_variant_mask(out["variant_mask"])
        L.oqp_set_lds_split(out["lds_split"])
    return out


if __name__ == "__main__":
    import json

    print(json.dumps(tune(), indent=1))
