#!/usr/bin/env python3
"""Benchmark: batched OCP-QP solves per second on one MI355X.

Workload (the headline value): 1024 same-size mass-spring QPs (8 masses:
nx=16, nu=7, N=30, dt=0.2, Q=I, R=0.1 I, |u|<=0.5, |x_pos|<=4, x0 ~
U[-2,2]^16 per instance), synthetic and seeded, resident in HBM before the
timed region.  One step = one full IPM solve of the whole batch (cold start
to the KKT tolerance), FP64 path; the mixed path is timed beside it.  Four
copies of the batch, each on its own stream and hardware queue, take the
steps in turn (--inflight): a batch is done only when its slowest instance
is (an infeasible instance runs 42 iterations where the others stop at
12-15), and the next batches fill the CUs its finished instances leave idle.
`one_batch_at_a_time` on the same line is the rate when every step waits for
the previous one; the roofline is that of single launches.

Further legs on the same line (context, not the headline):
  * pcond: the same batch solved through partial condensing to a shorter
    horizon (condensing and expansion inside the timed solve); N2 = 1 is full
    condensing, solved by the wide-stage kernel (dense Cholesky of the
    condensed Hessian);
  * abs: the same batch in the absolute formulation (mode speed_abs);
  * robust: the same batch with the QR-based factorization (mode robust);
  * balance: the same batch with checked Cholesky factors and the QR-based
    factorization as fallback (mode balance);
  * warm: the next receding-horizon problem of every solved instance, cold
    and warm-started from the shifted solution (warm_soft: the same with soft
    position boxes, slacks in the guess);
  * soft: the same batch with soft position boxes (every instance
    solvable), the same with and without slacks on the block kernel (the
    cost of the slack elimination), and the uneven batch with its first x0
    draws and soft state boxes;
  * uneven: a batch of random stable OCP QPs with nx ~ U{4..48},
    nu ~ U{1..16}, N ~ U{10..100} (one-wave variants plus the block kernel);
  * large: 256 large-stage QPs (nx = 128, nu = 32, N = 50, 32 general rows
    per stage; the block kernel's global-memory mode), FP64 to 1e-8 and
    mixed, one batch at a time and two batches in flight;
  * serve: the continuous-batching server replaying Poisson arrivals over a
    pool of uneven instances: saturated throughput at the offered rate, then
    p50/p99 latency at a sustainable rate, for the grouped FP64 and mixed
    paths and the plain per-request FP64 path (one launch per request), and
    the grouped FP64 path offered its saturated throughput as a steady stream
    (the largest sustained rate).

Prints one JSON line with the metric, the roofline of the dominant kernel
(algorithmic bytes / kernel time from HIP events on the launch stream) and
the CPU oracle timed on the host cores on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "OCP-QP solves/sec at KKT res <=1e-6 (batched, 1 GPU); p50/p99 serve latency"
HBM_PEAK_GBS = 8000.0
KKT_OK = 1e-6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


KERNEL_SOURCES = {
    # family -> (sources under csrc/, one-wave compile flags)
    "wave": (("ipm_kernel.h", "dev_common.h", "layout.h"), True),
    "block": (("ipm_block.h", "dev_common.h", "layout.h"), False),
    "batch": (("ipm_kernel.h", "ipm_block.h", "dev_common.h", "layout.h"), True),
}


def kernel_source_hash(family="wave"):
    """Hash of a kernel family's sources and compile flags: the one-wave
    kernel, the block kernel, or a whole batch solve (both kernels)."""
    from paper_2003_02547_amd import build as _build
    files, one_wave = KERNEL_SOURCES[family]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2003_02547_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(_build.FLAGS + (_build.ONE_WAVE_FLAGS if one_wave else [])).encode())
    return h.hexdigest()[:16]


def traffic_from_profile(key):
    """HBM bytes per launch (per batch solve for a whole-batch record) from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    rec = t.get(key)
    if not rec or rec.get("kernel_hash") != kernel_source_hash(rec.get("family", "wave")):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(qps, seconds, tol, single_qp=None):
    """The oracle, unmodified, on the host cores over the same instances; with
    single_qp also its one-thread time on that instance (the single-instance
    latency leg's CPU reference)."""
    import concurrent.futures as cf
    from oracle import oracle as O

    single = None
    if single_qp is not None:
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < 1.0:
            o = O.solve(single_qp, O.Arg.with_tol(1e-8))
            n += 1
        single = {"oracle_1thread_us": round((time.perf_counter() - t0) / n * 1e6, 1), "oracle_iters": int(o.iters)}

    threads = max(1, min(16, os.cpu_count() or 1))
    arg = O.Arg.with_tol(tol)
    t0 = time.perf_counter()

    refs = {}

    def work(k):
        cnt, i = 0, k
        while time.perf_counter() - t0 < seconds:
            j = i % len(qps)
            r = O.solve(qps[j], arg)
            cnt += int(r.status == O.SUCCESS)
            refs.setdefault(j, r)
            i += threads
        return cnt

    with cf.ThreadPoolExecutor(threads) as ex:
        total = sum(ex.map(work, range(threads)))
    el = time.perf_counter() - t0
    out = {"value": total / el, "unit": "solves/s", "cores": threads, "kind": "oracle",
           "sample": f"{total} instances of the same workload (round-robin over the batch), "
                     f"{threads} threads, one instance per thread at a time, {el:.1f} s"}
    if single is not None:
        out["single_instance"] = single
    return out, refs


def host_check(qps, refs, runs, large, large_picks):
    """Check the returned points on the host (the benchmark's CPU-baseline
    leg, the one place it runs the oracle): the KKT residual of every point,
    evaluated in FP64 by the oracle's residual routine, and the primal error
    against the oracle's solution, rel_err = |y - y_ref|_inf / max(1,
    |y_ref|_inf), over the instances the timed oracle sample solved (every
    instance when the sample covers the batch); for the large-stage batch on
    a few instances solved by the oracle here (FP64 with refinement, 1e-8)."""
    import concurrent.futures as cf

    import numpy as np
    from oracle import oracle as O

    threads = max(1, min(16, os.cpu_count() or 1))

    def err(sol, ref):
        y = np.concatenate([sol["u"], sol["x"]])
        yr = np.concatenate([ref["u"], ref["x"]])
        return float(np.max(np.abs(y - yr)) / max(1.0, np.max(np.abs(yr))))

    def summarize(qs, res, rf):
        with cf.ThreadPoolExecutor(threads) as ex:
            kkt = list(ex.map(lambda i: O.kkt_res(qs[i], res[i].sol), range(len(qs))))
        ok = [i for i in range(len(qs)) if res[i].status == 0 and kkt[i] <= KKT_OK]
        errs = [err(res[i].sol, rf[i].sol) for i in ok if i in rf and rf[i].status == O.SUCCESS]
        return {"solves_ok_host": len(ok), "max_kkt_res_host": float(max(kkt[i] for i in ok)) if ok else None,
                "rel_err_max": float(max(errs)) if errs else None,
                "rel_err_p50": float(np.median(errs)) if errs else None, "compared": len(errs)}

    out = {"kkt": "oracle residual routine, FP64, every returned point",
           "rel_err": "|y - y_ref|_inf / max(1, |y_ref|_inf) against the oracle's FP64 solution at 1e-8"}
    for name, res in runs.items():
        out[name] = summarize(qps, res, refs)
    if large is not None and large_picks > 0:
        lq, lres = large
        picks = list(range(0, len(lq), max(1, len(lq) // large_picks)))[:large_picks]
        arg = O.Arg.with_tol(1e-8, ir_max=4)
        with cf.ThreadPoolExecutor(threads) as ex:
            lrefs = dict(zip(picks, ex.map(lambda i: O.solve(lq[i], arg), picks)))
        out["large"] = {name: summarize(lq, res, lrefs) for name, res in lres.items()}
        out["large"]["oracle_sample"] = picks
    return out


def leg_uneven(B, W, torch, np, count, steps, pool, seed0=0):
    """Uneven batch: every instance solved in one batch solve, one launch per
    kernel group, the groups spread over the batch stream and 3 extra
    streams (and, for comparison, all on the batch stream)."""
    from paper_2003_02547_amd import perfmodel
    qps = [W.random_uneven(seed0 + i) for i in range(count)]
    dbytes = np.array([perfmodel.data_bytes(q) for q in qps], dtype=np.float64)
    fpi = np.array([perfmodel.flops_per_iter(q) for q in qps], dtype=np.float64)
    out = {}
    for name, mode, streams in (("f64", B.MODE_F64, pool), ("mixed", B.MODE_MIXED, pool), ("f64_one_stream", B.MODE_F64, 0)):
        batch = B.Batch(qps, B.default_arg(mode), streams=streams).load().sync()
        batch.solve()
        torch.cuda.synchronize()
        st = batch.stream
        ms = []
        for _ in range(steps):
            s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s_.record(st)
            batch.solve()
            e_.record(st)
            torch.cuda.synchronize()
            ms.append(s_.elapsed_time(e_))
        batch.fetch().sync()
        stats = [batch.stat(i) for i in range(count)]
        ok = sum(1 for x in stats if x.status == B.SUCCESS and max(x.res[:]) <= KKT_OK)
        groups = sorted({batch.variant(i)[0] for i in range(count)})
        nv = B.lib().oqp_variant_count()
        t = float(np.median(ms)) * 1e-3
        nres = np.array([x.iters + 1 + x.ir_steps for x in stats])
        its = np.array([x.iters for x in stats])
        alg = float(np.sum(dbytes * nres))
        ach = alg / t / 1e9
        tkey = "uneven_%d_%s_batch" % (count, name) if seed0 == 0 else None
        out[name] = {"value": round(ok / t, 1), "unit": "solves/s",
                     "ms_per_step": round(t * 1e3, 3), "solves_ok": ok,
                     "block_kernel_instances": sum(1 for i in range(count) if batch.variant(i)[0] >= nv),
                     "kernel_groups": len(groups), "extra_streams": len(streams) if isinstance(streams, list) else streams,
                     "roofline": {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(ach / HBM_PEAK_GBS, 5),
                                  "traffic": traffic_from_profile(tkey) if tkey else None,
                                  "alg_bytes": alg,
                                  "scope": "whole batch solve (every kernel group), batch-stream events",
                                  "fp64_tflops": round(float(np.sum(fpi * its)) / t / 1e12, 4)}}
        del batch
    out["instances"] = count
    out["sizes"] = "nx~U{4..48}, nu~U{1..16}, N~U{10..100}, boxes on all u and x"
    return out


def leg_pcond(B, W, torch, np, qps, n2s, steps):
    """The headline batch solved through partial condensing (Section 3.5) to
    N2 stages: condensing, IPM on the condensed QPs and expansion, all inside
    each timed solve.  A solve counts when the condensed solve reports success
    with residual norms within the KKT tolerance."""
    out = {}
    for N2 in n2s:
        batch = B.Batch(qps, B.default_arg(cond_N=N2)).load().sync()
        batch.solve()
        torch.cuda.synchronize()
        st = batch.stream
        ms = []
        for _ in range(steps):
            s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s_.record(st)
            batch.solve()
            e_.record(st)
            torch.cuda.synchronize()
            ms.append(s_.elapsed_time(e_))
        batch.fetch().sync()
        stats = [batch.stat(i) for i in range(len(qps))]
        ok = sum(1 for x in stats if x.status == B.SUCCESS and max(x.res[:]) <= KKT_OK)
        iters = np.array([x.iters for x in stats])
        v, dims = batch.variant(0)
        med = float(np.median(ms))
        out[str(N2)] = {"value": round(ok / (med * 1e-3), 1), "unit": "solves/s", "ms_per_step": round(med, 3),
                        "solves_ok": ok, "iters_p50": float(np.percentile(iters, 50)),
                        "iters_p99": float(np.percentile(iters, 99)), "kernel_group": v,
                        "stage_sizes_padded": list(dims)}
        del batch
    return out


def leg_warm(B, W, torch, np, qps, steps):
    """Receding horizon on the headline batch: after a cold solve, the next
    problem of every solved instance (x_0 <- x_1) is solved cold and
    warm-started (primal-dual guess, Section 4.2) from the shifted solution.
    The guess upload is inside the timed solve; building it on the host is
    not."""
    first = B.Batch(qps, B.default_arg()).load().solve().fetch().sync()
    res = first.results()
    del first
    keep = [i for i, r in enumerate(res) if r.status == B.SUCCESS]
    pairs = [W.receding_step(qps[i], res[i].sol) for i in keep]
    nxt, guesses = [p[0] for p in pairs], [p[1] for p in pairs]
    out = {"instances": len(nxt)}
    for name, warm in (("cold", 0), ("warm", 2)):
        b = B.Batch(nxt, B.default_arg(warm_start=warm)).load().sync()
        ms = []
        for step in range(steps + 1):
            if warm:
                for i, g in enumerate(guesses):
                    b.set_iterate(i, g)
            torch.cuda.synchronize()
            s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s_.record(b.stream)
            b.solve()
            e_.record(b.stream)
            torch.cuda.synchronize()
            if step > 0:
                ms.append(s_.elapsed_time(e_))
        b.fetch().sync()
        stats = [b.stat(i) for i in range(len(nxt))]
        ok = sum(1 for x in stats if x.status == B.SUCCESS and max(x.res[:]) <= KKT_OK)
        iters = np.array([x.iters for x in stats])
        med = float(np.median(ms))
        out[name] = {"value": round(ok / (med * 1e-3), 1), "unit": "solves/s", "ms_per_step": round(med, 3),
                     "solves_ok": ok, "iters_p50": float(np.percentile(iters, 50)), "iters_max": int(iters.max()),
                     "iters_mean": round(float(iters.mean()), 2)}
        del b
    return out


def leg_abs(B, torch, np, qps, steps):
    """The headline batch in the absolute formulation (mode speed_abs: no
    residuals in the loop, exit on the duality measure, residual norms of
    the returned point reported).  Cancellation near the solution keeps its
    residuals above the delta path's, so it is reported with both counts: the
    solves that exit on the duality measure and those that also meet the KKT
    tolerance."""
    b = B.Batch(qps, B.default_arg(B.MODE_ABS)).load().sync()
    b.solve()
    torch.cuda.synchronize()
    ms = []
    for _ in range(steps):
        s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s_.record(b.stream)
        b.solve()
        e_.record(b.stream)
        torch.cuda.synchronize()
        ms.append(s_.elapsed_time(e_))
    b.fetch().sync()
    stats = [b.stat(i) for i in range(len(qps))]
    exit_ok = sum(1 for x in stats if x.status == B.SUCCESS)
    kkt_ok = sum(1 for x in stats if x.status == B.SUCCESS and max(x.res[:]) <= KKT_OK)
    iters = np.array([x.iters for x in stats])
    res = np.array([max(x.res[:]) for x in stats if x.status == B.SUCCESS])
    med = float(np.median(ms))
    del b
    return {"ms_per_step": round(med, 3), "exit_on_mu": exit_ok, "kkt_ok": kkt_ok,
            "value_exit_on_mu": round(exit_ok / (med * 1e-3), 1), "unit": "solves/s",
            "iters_p50": float(np.percentile(iters, 50)), "iters_max": int(iters.max()),
            "kkt_res_p50": float(np.median(res)) if res.size else None, "tol_comp_on_mu": 1e-8}


def leg_robust(B, torch, np, qps, steps, mode=None):
    """The headline batch with the QR-based factorization (mode robust):
    same iterations as the Cholesky path, factors from an array algorithm,
    refinement of the prediction-centering-correction direction; or (mode
    balance) with Cholesky factors checked by the predictor's refinement
    residual and refactored with the array algorithm when the check fails."""
    mode = B.MODE_ROBUST if mode is None else mode
    b = B.Batch(qps, B.default_arg(mode)).load().sync()
    b.solve()
    torch.cuda.synchronize()
    ms = []
    for _ in range(steps):
        s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s_.record(b.stream)
        b.solve()
        e_.record(b.stream)
        torch.cuda.synchronize()
        ms.append(s_.elapsed_time(e_))
    b.fetch().sync()
    stats = [b.stat(i) for i in range(len(qps))]
    ok = sum(1 for x in stats if x.status == B.SUCCESS and max(x.res[:]) <= KKT_OK)
    iters = np.array([x.iters for x in stats])
    med = float(np.median(ms))
    del b
    return {"value": round(ok / (med * 1e-3), 1), "unit": "solves/s", "ms_per_step": round(med, 3), "solves_ok": ok,
            "iters_p50": float(np.percentile(iters, 50)), "iters_max": int(iters.max()),
            "ir_steps": int(sum(x.ir_steps for x in stats)), "qr_refactors": int(sum(x.qr_refactors for x in stats))}


def _median_solve_ms(b, torch, np, steps):
    """Median time of `steps` solves of a loaded batch (one untimed solve
    first), HIP events on the batch stream; fetches the last results."""
    b.solve()
    torch.cuda.synchronize()
    ms = []
    for _ in range(steps):
        s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s_.record(b.stream)
        b.solve()
        e_.record(b.stream)
        torch.cuda.synchronize()
        ms.append(s_.elapsed_time(e_))
    b.fetch().sync()
    return float(np.median(ms))


def leg_soft(B, W, torch, np, qps, steps, uneven_count, uneven_steps, pool):
    """Soft constraints (Section 2.2): the headline batch with its position
    boxes soft (per slack an L2 weight of 1 and an L1 weight of 10), which
    makes every instance solvable, on the kernels the batch picks (the
    one-wave kernel's soft build); the cost of the slack elimination within
    one kernel family, as the same two batches (with and without slacks) on
    the block kernel; then the uneven batch with its first x0 draws (no
    redraw for a feasible zero-input rollout) and soft state boxes."""
    out = {"weights": f"state boxes after stage 0 soft, Z={W.SOFT_Z}, z={W.SOFT_z} per slack", "tol": 1e-8}

    def summary(b, n, med):
        stats = [b.stat(i) for i in range(n)]
        ok = sum(1 for x in stats if x.status == B.SUCCESS and max(x.res[:]) <= KKT_OK)
        iters = np.array([x.iters for x in stats])
        return {"value": round(ok / (med * 1e-3), 1), "unit": "solves/s", "ms_per_step": round(med, 3),
                "solves_ok": ok, "instances": n, "iters_p50": float(np.percentile(iters, 50)),
                "iters_max": int(iters.max())}

    sq = [W.mass_spring_chain8_soft(i) for i in range(len(qps))]
    b = B.Batch(sq, B.default_arg()).load().sync()
    r = summary(b, len(sq), _median_solve_ms(b, torch, np, steps))
    sols = [b.solution(i) for i in range(len(sq))]
    r["slack_active"] = sum(1 for x in sols if max(x["s_l"].max(), x["s_u"].max()) > 1e-6)
    v, (nx, nu, ng) = b.variant(0)
    r["kernel"] = f"ipm_kernel<{nx},{nu},{ng}> soft build"
    out["chain8"] = r
    del b
    L = B.lib()
    wmax = L.oqp_get_wave_max()
    L.oqp_set_wave_max(0)  # every instance on the block kernel
    try:
        for key, batch in (("chain8_block_soft", sq), ("chain8_block_f64_no_slacks", qps)):
            b = B.Batch(batch, B.default_arg()).load().sync()
            out[key] = summary(b, len(batch), _median_solve_ms(b, torch, np, steps))
            del b
    finally:
        L.oqp_set_wave_max(wmax)
    if uneven_count > 0:
        uq = [W.random_uneven_soft(i) for i in range(uneven_count)]
        b = B.Batch(uq, B.default_arg(), streams=pool).load().sync()
        r = summary(b, len(uq), _median_solve_ms(b, torch, np, uneven_steps))
        r["first_draw_infeasible_hard"] = sum(1 for i in range(uneven_count) if W.random_uneven(i).meta["redraws"] > 0)
        r["extra_streams"] = 3
        out["uneven"] = r
        del b
    return out


def leg_single(B, W, torch, np, reps):
    """Latency of one 4-mass QP (nx = 8, nu = 3, N = 10, dt = 0.5; seed 1) in
    a batch of one: one launch, FP64 to 1e-8, median over reps (the CPU
    baseline times the oracle on the same instance)."""
    qp = W.mass_spring_chain4(1)
    batch = B.Batch([qp], B.default_arg()).load().sync()
    batch.solve()
    torch.cuda.synchronize()
    st = batch.stream
    ms = []
    for _ in range(reps):
        s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s_.record(st)
        batch.solve()
        e_.record(st)
        torch.cuda.synchronize()
        ms.append(s_.elapsed_time(e_))
    batch.fetch().sync()
    r = batch.result(0)
    return {"workload": "mass_spring_4masses_N10", "gpu_us_p50": round(float(np.median(ms)) * 1e3, 1),
            "iters": int(r.iters), "status": int(r.status)}


def leg_large(B, W, torch, np, perfmodel, count, steps, pool, inflight=2):
    """Large-stage batch (nx = 128, nu = 32, N = 50, 32 general rows per
    stage): the block kernel's global-memory mode.  FP64 to the FP64 bar
    (KKT 1e-8) with up to 4 refinement corrections of the
    prediction-centering-correction direction (without them the iteration
    stalls before 1e-8 on some instances, in the oracle as well); mixed to the
    metric's 1e-6.  Roofline: algorithmic flops of the method (factorization,
    two solves and one residual per iteration, one solve and one residual per
    refinement correction) over the launch time, against the FP64 matrix-core
    peak (FP32 for the mixed path's factorization).  `inflight` copies of the
    batch on the pool's streams then take the steps together: one batch puts
    one workgroup on each CU, two fill both wave slots of every SIMD."""
    qps = [W.random_large_stage(i) for i in range(count)]
    fpi = np.array([perfmodel.flops_per_iter(q) for q in qps])
    fir = np.array([perfmodel.flops_per_refinement(q) for q in qps])
    dbytes = np.array([perfmodel.data_bytes(q) for q in qps], dtype=np.float64)
    out = {"instances": count, "sizes": "nx=128, nu=32, N=50, ng=32 (C=0)"}
    keep = {}
    for name, mode, tol, irm in (("f64", B.MODE_F64, 1e-8, 4), ("mixed", B.MODE_MIXED, KKT_OK, 4)):
        arg = B.default_arg(mode, tol_stat=tol, tol_eq=tol, tol_ineq=tol, tol_comp=tol, ir_max=irm)
        batch = B.Batch(qps, arg).load().sync()
        batch.solve()
        torch.cuda.synchronize()
        st = batch.stream
        ms = []
        for _ in range(steps):
            s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s_.record(st)
            batch.solve()
            e_.record(st)
            torch.cuda.synchronize()
            ms.append(s_.elapsed_time(e_))
        batch.fetch().sync()
        res = batch.results()
        ok = sum(1 for x in res if x.status == B.SUCCESS and max(x.res[:]) <= KKT_OK)
        its = np.array([x.iters for x in res])
        irs = np.array([x.ir_steps for x in res])
        t = float(np.median(ms)) * 1e-3
        flops = float(np.sum(fpi * its + fir * irs))
        fell = sum(1 for x in res if x.fell_back_f64)
        peak = 78.6 if mode == B.MODE_F64 else 157.3
        ach = flops / t / 1e12
        del batch
        # the same batch, `inflight` copies at once
        nb, tw, same = 1, t, True
        if inflight > 1:
            copies = [B.Batch(qps, arg, stream=st).load().sync() for st in pool[:inflight]]
            nb = len(copies)
            for c in copies:
                c.solve()
            torch.cuda.synchronize()
            walls = []
            for _ in range(steps):
                t0 = time.perf_counter()
                for c in copies:
                    c.solve()
                torch.cuda.synchronize()
                walls.append(time.perf_counter() - t0)
            for c in copies:
                c.fetch().sync()
                for a, x in zip(c.results(), res):
                    same = same and a.status == x.status and a.iters == x.iters and bool(
                        np.array_equal(a.sol["u"], x.sol["u"], equal_nan=True))
            del copies
            tw = float(np.median(walls))
        out[name] = {"value": round(nb * ok / tw, 1), "unit": "solves/s",
                     "ms_per_step": round(tw * 1e3, 3), "batches_in_flight": nb,
                     "inflight_results_equal": same,
                     "one_batch_at_a_time": {"value": round(ok / t, 1), "ms_per_step": round(t * 1e3, 3)},
                     "solves_ok": ok, "tol": tol, "ir_max": irm,
                     "non_success": [i for i, x in enumerate(res) if x.status != B.SUCCESS],
                     "iters_p50": float(np.median(its)), "iters_max": int(its.max()),
                     "ir_steps_mean": round(float(irs.mean()), 2), "fell_back_f64": fell,
                     "max_kkt_res_kernel": float(max(max(x.res[:]) for x in res)),
                     "roofline": {"bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
                                  "frac": round(ach / peak, 5),
                                  "traffic": traffic_from_profile("ipm_block_kernel<0,256,64>")
                                  if mode == B.MODE_F64 and count == 256 else None,
                                  "alg_flops": flops,
                                  "kernel": "ipm_block_kernel<%d,256,64>" % (0 if mode == B.MODE_F64 else 1),
                                  "hbm_gbs": round(float(np.sum(dbytes * (its + 1 + irs))) / t / 1e9, 1),
                                  "scope": "one batch at a time (launch time)",
                                  "frac_in_flight": round(nb * flops / tw / 1e12 / peak, 5)}}
        keep[name] = res
    return out, qps, keep


def leg_serve(B, W, torch, np, pool_n, offered, sat_seconds, sus_frac, sus_seconds, per_req_seconds, log,
              iter_block=4, nstreams=5):
    """Continuous-batching server, native real-time replay of Poisson
    arrivals over a pool of pre-packed uneven instances (page-locked host
    memory; each request's data is uploaded on admission); also the same
    pool with first x0 draws and soft state boxes."""
    pool = [W.random_uneven(100000 + i) for i in range(pool_n)]
    packed = [B.Packed(q, pinned=True) for q in pool]
    # the same draws with their first x0 and soft state boxes (no redraw)
    packed_soft = [B.Packed(W.random_uneven_soft(100000 + i), pinned=True) for i in range(pool_n)]
    dev_bytes = int(min(64 << 30, 2 * sum(p.footprint for p in packed_soft) + (1 << 30)))
    tol = dict(tol_stat=KKT_OK, tol_eq=KKT_OK, tol_ineq=KKT_OK, tol_comp=KKT_OK)

    def run(mode, max_launch, rate, seconds, seed, pk=None, iter_block=0):
        pk = packed if pk is None else pk
        srv = B.Server(B.default_arg(mode, **tol), dev_bytes=dev_bytes, nstreams=nstreams, max_launch=max_launch,
                       max_requests=4096, max_groups=1024, iter_block=iter_block)
        try:
            times, idx = W.serving_stream(rate, seconds, pool_n, seed=seed)
            lat, stats, wall = srv.replay([pk[i] for i in idx], times, timeout=120.0)
            c = srv.stats()
        finally:
            srv.close()
        ok = sum(1 for x in stats if x.status == B.SUCCESS)
        return {"offered_per_s": rate, "requests": len(times), "served_per_s": round(ok / wall, 1),
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3), "launches": int(c["launches"]),
                "dev_peak_mb": round(c["dev_peak"] / 2**20, 1), "wall_s": round(wall, 2)}

    log(f"bench: serve warm-up and saturation at {offered:.0f} req/s offered")
    run(B.MODE_F64, 256, offered, 0.05, 1)
    sat = run(B.MODE_F64, 256, offered, sat_seconds, 2)
    rate = max(10.0, round(sus_frac * sat["served_per_s"], -1))
    out = {"pool": pool_n, "saturated_f64": sat, "sustained_rate_per_s": rate}
    # iteration blocks: launches of at most `iter_block` IPM iterations, new
    # arrivals join unfinished requests at the block boundaries
    log(f"bench: serve saturation with iteration blocks of {iter_block}")
    out["iter_block"] = iter_block
    out["saturated_f64_blocks"] = run(B.MODE_F64, 256, offered, sat_seconds, 2, iter_block=iter_block)
    for name, mode, ml in (("f64", B.MODE_F64, 256), ("mixed", B.MODE_MIXED, 256)):
        log(f"bench: serve {name} at {rate:.0f} req/s for {sus_seconds:.0f} s")
        out[name] = run(mode, ml, rate, sus_seconds, 3)
    log(f"bench: serve f64 with iteration blocks at {rate:.0f} req/s for {sus_seconds:.0f} s")
    out["f64_blocks"] = run(B.MODE_F64, 256, rate, sus_seconds, 3, iter_block=iter_block)
    # the largest sustained rate: the saturated throughput offered as a
    # steady Poisson stream (latency stays bounded when it is sustained)
    top = max(10.0, round(sat["served_per_s"], -1))
    out["sustained_max_rate_per_s"] = top
    log(f"bench: serve f64 at the saturated rate, {top:.0f} req/s for {sus_seconds:.0f} s (plain and in iteration blocks)")
    out["f64_at_saturated_rate"] = run(B.MODE_F64, 256, top, sus_seconds, 4)
    out["f64_blocks_at_saturated_rate"] = run(B.MODE_F64, 256, top, sus_seconds, 4, iter_block=iter_block)
    log(f"bench: serve f64 with soft state boxes (first x0 draws) at {rate:.0f} req/s for {sus_seconds:.0f} s")
    out["f64_soft"] = run(B.MODE_F64, 256, rate, sus_seconds, 3, packed_soft)
    # plain per-request FP64 path (one launch per request): same offered rate
    # over a shorter window, since it saturates far below that rate
    log(f"bench: serve f64_per_request at {rate:.0f} req/s for {per_req_seconds:.2f} s")
    out["f64_per_request"] = run(B.MODE_F64, 1, rate, per_req_seconds, 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--instances", type=int, default=1024)
    ap.add_argument("--mode", choices=["f64"], default="f64")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--uneven", type=int, default=4096, help="instances of the uneven leg (0: skip)")
    ap.add_argument("--uneven-steps", type=int, default=3)
    ap.add_argument("--inflight", type=int, default=4,
                    help="copies of the headline batch solved in turn on their own streams (1: one at a time): the "
                         "three pool streams, then the default stream; the process has four hardware queues "
                         "(measured: 3 in flight 116k/s, 4 in flight 124k/s; 4 on four new streams, two of them "
                         "sharing a queue, 78k/s)")
    ap.add_argument("--pcond", default="1,5,10,15", help="condensed horizons for the partial-condensing leg (0: skip)")
    ap.add_argument("--pcond-steps", type=int, default=5)
    ap.add_argument("--warm-steps", type=int, default=5, help="timed solves of the warm-start leg (0: skip)")
    ap.add_argument("--abs-steps", type=int, default=5, help="timed solves of the absolute-formulation leg (0: skip)")
    ap.add_argument("--robust-steps", type=int, default=5, help="timed solves of the QR-factorization leg (0: skip)")
    ap.add_argument("--iter20-steps", type=int, default=5, help="timed solves of the iter_max 20 context line (0: skip)")
    ap.add_argument("--soft-steps", type=int, default=5, help="timed solves of the soft-constraint leg (0: skip)")
    ap.add_argument("--soft-uneven", type=int, default=4096, help="instances of the soft uneven batch (0: skip)")
    ap.add_argument("--large", type=int, default=256, help="instances of the large-stage leg (0: skip)")
    ap.add_argument("--large-steps", type=int, default=2)
    ap.add_argument("--large-inflight", type=int, default=2,
                    help="copies of the large-stage batch solved at once (at most 3, the pool's streams)")
    ap.add_argument("--large-check", type=int, default=16,
                    help="large-stage instances the host check solves with the oracle for the primal error")
    ap.add_argument("--serve-pool", type=int, default=256, help="distinct instances in the serving pool (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=20000.0, help="offered Poisson rate for the saturation run")
    ap.add_argument("--serve-sat-seconds", type=float, default=0.25)
    ap.add_argument("--serve-frac", type=float, default=0.5, help="sustained rate as a fraction of saturated throughput")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--serve-per-request-seconds", type=float, default=0.2)
    ap.add_argument("--serve-streams", type=int, default=5,
                    help="server streams (one for solution fetches, the rest for launches)")
    ap.add_argument("--serve-iter-block", type=int, default=4,
                    help="IPM iterations per launch in the iteration-block serving runs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        sys.exit("bench.py: the benchmark runs on one GPU only (--gpus 1); instances are independent, "
                 "and a multi-GPU run would shard the batch by estimated cost with no exchange.")

    import numpy as np
    import torch

    if args.calibrate_copy:
        torch.cuda.set_device(0)
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": n, "copies": 3}), flush=True)
        return

    from paper_2003_02547_amd import binding as B
    from paper_2003_02547_amd import perfmodel, workloads as W

    torch.cuda.set_device(0)
    # one fixed set of extra streams (default priority), created before any
    # other, for every leg that runs work concurrently: the process has four
    # hardware queues, one of them the default stream's, and streams created
    # later may share a queue with the default stream, which serializes the
    # work put on the two
    pool = [torch.cuda.Stream() for _ in range(3)]
    log(f"bench: generating {args.instances} mass-spring QPs (nx=16, nu=7, N=30)")
    qps = [W.mass_spring_chain8(i) for i in range(args.instances)]
    dbytes = np.array([perfmodel.data_bytes(q) for q in qps], dtype=np.float64)
    fpi = np.array([perfmodel.flops_per_iter(q) for q in qps], dtype=np.float64)

    def time_path(mode, steps, warmup, inflight=1, **over):
        """Solve the batch `steps` times.  inflight > 1: that many copies of
        the batch, each on its own stream (default priority), take the steps
        in turn, so a batch whose instances are mostly done shares the GPU
        with the next one instead of leaving it idle behind its slowest
        instance; every copy solves every instance of every step in full."""
        arg = B.default_arg(mode, **over)
        if inflight > 1:
            # the pool's streams first, then the default stream (the fourth
            # hardware queue), then new streams (sharing queues)
            streams = (pool + [torch.cuda.current_stream()])[:inflight]
            streams += [torch.cuda.Stream() for _ in range(inflight - len(streams))]
            batches = [B.Batch(qps, arg, stream=st) for st in streams]
        else:
            batches = [B.Batch(qps, arg)]
        for bt in batches:
            bt.load().sync()
        batch = batches[0]
        variant = batch.variant(0)[1]
        for w in range(max(warmup, len(batches) if warmup > 0 else 0)):
            batches[w % len(batches)].solve()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k, (s_, e_) in enumerate(ev):
            bt = batches[k % len(batches)]
            s_.record(bt.stream)
            bt.solve()
            e_.record(bt.stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kern_ms = np.array([s_.elapsed_time(e_) for s_, e_ in ev])
        for bt in batches:
            bt.fetch().sync()
        res = batch.results()
        same = True
        for bt in batches[1:]:
            for i, r in enumerate(bt.results()):
                same = same and r.status == res[i].status and r.iters == res[i].iters and bool(
                    np.array_equal(r.sol["u"], res[i].sol["u"], equal_nan=True))
        status = np.array([r.status for r in res])
        kkt = np.array([float(np.max(r.res)) for r in res])
        iters = np.array([r.iters for r in res])
        irs = np.array([r.ir_steps for r in res])
        fb = np.array([r.fell_back_f64 for r in res])
        ok = int(np.sum((status == B.SUCCESS) & (kkt <= KKT_OK)))
        wall = t1 - t0
        kern_s = float(np.mean(kern_ms)) * 1e-3
        nres = iters + 1 + irs  # residual evaluations: one per iteration, the final check, one per refinement
        alg_bytes = float(np.sum(dbytes * nres))
        return dict(variant=variant, ok=ok, wall=wall, steps=steps, kern_ms=kern_ms, kern_s=kern_s,
                    status=status, kkt=kkt, iters=iters, irs=irs, fb=fb, res=res, alg_bytes=alg_bytes,
                    achieved=alg_bytes / kern_s / 1e9, flops=float(np.sum(fpi * iters)) / kern_s / 1e12,
                    value=ok * steps / wall, same=same, del_batch=batches)

    log(f"bench: FP64 path, warmup {args.warmup}, {args.steps} steps, one batch at a time")
    f = time_path(B.MODE_F64, args.steps, args.warmup)
    fp = f
    if args.inflight > 1:
        log(f"bench: FP64 path, {args.inflight} batches in flight, warmup {args.warmup}, {args.steps} steps")
        fp = time_path(B.MODE_F64, args.steps, args.warmup, inflight=args.inflight)
    log(f"bench: mixed path, warmup {args.warmup}, {args.steps} steps")
    m = time_path(B.MODE_MIXED, args.steps, args.warmup)
    f20 = None
    if args.iter20_steps > 0:
        log("bench: FP64 path with iter_max 20 (context: the batch time follows its slowest instance)")
        f20 = time_path(B.MODE_F64, args.iter20_steps, 1, iter_max=20)
    vkey = "ipm_kernel<%d,%d,%d>" % f["variant"]
    traffic = traffic_from_profile(vkey)
    okmask = f["status"] == B.SUCCESS
    line = {
        "metric": METRIC,
        "value": round(fp["value"], 1),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * fp["wall"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "mass_spring_8masses_x1024", "instances": args.instances, "nx": 16, "nu": 7,
                   "N": 30, "path": "f64", "kernel": vkey, "batches_in_flight": args.inflight},
        "one_batch_at_a_time": {"value": round(f["value"], 1), "unit": "solves/s",
                                "ms_per_step": round(1e3 * f["wall"] / args.steps, 4),
                                "note": "each step waits for the previous batch's slowest instance"},
        "inflight_results_equal": bool(fp["same"]) and (fp is f or bool(
            np.array_equal(fp["status"], f["status"]) and np.array_equal(fp["iters"], f["iters"]))),
        "roofline": {"bound": "hbm", "achieved": round(f["achieved"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(f["achieved"] / HBM_PEAK_GBS, 5), "traffic": traffic,
                     "alg_bytes": f["alg_bytes"]},
        "kernel_ms": round(float(np.mean(f["kern_ms"])), 4),
        "fp64_tflops": round(f["flops"], 4),
        "solves_ok": f["ok"],
        "non_success": int(np.sum(~okmask)),
        "iters_p50": float(np.percentile(f["iters"], 50)),
        "iters_p99": float(np.percentile(f["iters"], 99)),
        "max_kkt_res": float(np.max(f["kkt"][okmask])) if okmask.any() else None,
        "latency_ms_p50": round(float(np.percentile(f["kern_ms"], 50)), 4),
        "latency_ms_p99": round(float(np.percentile(f["kern_ms"], 99)), 4),
        "mixed": {"value": round(m["value"], 1), "unit": "solves/s", "dtype": "f32 factor+sweeps, f64 pivots/residuals/refinement",
                  "ms_per_step": round(1e3 * m["wall"] / args.steps, 4), "solves_ok": m["ok"],
                  "iters_p50": float(np.percentile(m["iters"], 50)),
                  "ir_steps_mean": round(float(np.mean(m["irs"])), 2),
                  "fell_back_f64": int(np.sum(m["fb"])),
                  "max_kkt_res": float(np.max(m["kkt"][m["status"] == B.SUCCESS])),
                  "vs_f64": round(m["value"] / f["value"], 3)},
    }
    if f20 is not None:
        line["iter_max_20"] = {"value": round(f20["value"], 1), "unit": "solves/s",
                               "ms_per_step": round(1e3 * f20["wall"] / f20["steps"], 4), "solves_ok": f20["ok"],
                               "iters_max": int(np.max(f20["iters"]))}
        del f20["del_batch"]
    del f["del_batch"], m["del_batch"]
    fp.pop("del_batch", None)
    n2s = [int(x) for x in args.pcond.split(",") if x.strip() and int(x) > 0]
    if n2s:
        log(f"bench: partial condensing leg, N2 in {n2s}")
        line["pcond"] = leg_pcond(B, W, torch, np, qps, n2s, args.pcond_steps)
    if args.robust_steps > 0:
        log("bench: QR-based factorization (robust mode) leg")
        line["robust"] = leg_robust(B, torch, np, qps, args.robust_steps)
        log("bench: balance mode")
        line["balance"] = leg_robust(B, torch, np, qps, args.robust_steps, B.MODE_BALANCE)
    if args.abs_steps > 0:
        log("bench: absolute-formulation leg")
        line["abs"] = leg_abs(B, torch, np, qps, args.abs_steps)
    if args.warm_steps > 0:
        log("bench: receding-horizon warm-start leg")
        line["warm"] = leg_warm(B, W, torch, np, qps, args.warm_steps)
        log("bench: receding-horizon leg with soft position boxes")
        line["warm_soft"] = leg_warm(B, W, torch, np, [W.mass_spring_chain8_soft(i) for i in range(len(qps))],
                                     args.warm_steps)
    log("bench: single-instance latency (4 masses, N = 10)")
    line["single"] = leg_single(B, W, torch, np, 20)
    if args.soft_steps > 0:
        log("bench: soft-constraint leg")
        line["soft"] = leg_soft(B, W, torch, np, qps, args.soft_steps, args.soft_uneven, args.uneven_steps, pool)
    if args.uneven > 0:
        log(f"bench: uneven leg, {args.uneven} instances")
        line["uneven"] = leg_uneven(B, W, torch, np, args.uneven, args.uneven_steps, pool)
    large = None
    if args.large > 0:
        log(f"bench: large-stage leg, {args.large} instances")
        line["large"], lq, lres = leg_large(B, W, torch, np, perfmodel, args.large, args.large_steps, pool,
                                            args.large_inflight)
        large = (lq, lres)
    if args.serve_pool > 0:
        line["serve"] = leg_serve(B, W, torch, np, args.serve_pool, args.serve_rate, args.serve_sat_seconds,
                                  args.serve_frac, args.serve_seconds, args.serve_per_request_seconds, log,
                                  args.serve_iter_block, args.serve_streams)
    if not args.no_cpu_baseline:
        log(f"bench: CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        line["cpu_baseline"], refs = cpu_baseline(qps, args.cpu_seconds, 1e-8, W.mass_spring_chain4(1))
        log("bench: host check of the returned points against the oracle")
        chk = host_check(qps, refs, {"f64": f["res"], "mixed": m["res"]}, large, args.large_check)
        # the headline counts only solves whose KKT residual, evaluated on the
        # host in FP64, meets the metric's bound
        line["solves_ok_host"] = chk["f64"]["solves_ok_host"]
        line["value"] = round(chk["f64"]["solves_ok_host"] * args.steps / fp["wall"], 1)
        line["host_check"] = chk
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
