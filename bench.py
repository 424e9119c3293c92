#!/usr/bin/env python3
"""Benchmark: the whole subtraction on a 1e7-binary catalog on one MI355X.

A step is one gbsub_run (prep, every loop body until the resolved set stops
changing, outputs) over a catalog already resident in HBM.  Prints one JSON
line: binary-iterations/s (= sources x loop bodies / wall time of a run),
the roofline of the dominant kernel measured live with HIP events over the
timed steps, and the FP64 oracle timed on the host cores on a bounded
sample of the same workload.

  python bench.py [--gpus 1] [--steps 20] [--warmup 3]

Other workloads print one JSON line each:
  --workload batch   64 catalogs (N log-uniform in [1e5, 2e7], per-catalog
                     hyperparameters, T = 4 yr, W = 1001): catalogs/h through
                     one shared batch against the same catalogs run one by one;
  --workload serve   a Poisson stream of jobs (N log-uniform in [1e5, 3e7],
                     T in {1, 2, 4} yr) through the continuous-batching server:
                     p50/p99 latency at 0.7x the measured saturated rate;
  --workload precision   the 1e7-binary catalog in FP64, FP32 with compensated
                     sums and naive FP32: spectrum and SNR errors and resolve-
                     decision flips against the FP64 oracle's stored results;
  --workload generate    catalogs drawn on the GPU from the population model;
  --workload oracle      the FP64 oracle alone on the host cores (one thread
                     and all threads, 1e4 and 1e7 catalogs, a subset of the
                     64-catalog batch);
  --workload cx          the complex-template data model (gbsub_cx_run) on the
                     1e7-binary catalog with its channel phases.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s

# Algorithmic bytes per work unit of each kernel family (what the method must
# move, not what the implementation happens to move).
ALGO_BYTES = {
    "median": 24.0,    # per output bin: read X and S_instr, write S
    "xupdate": 24.0,   # per bin: read the 128-bit difference entry, write X
    "prep": 28.0,      # per source: read A, f, fdot; two 8-byte accumulator updates
    "snr": 36.0,       # per candidate evaluation: track, q, state, one S gather, write rho^2
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(kernel: str):
    """HBM bytes per working launch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, if it was taken on the current kernel
    source (else None: the counters no longer describe this build)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_1e7_traffic.json")
    try:
        with open(path) as fh:
            js = json.load(fh)
    except (OSError, ValueError):
        return None
    from paper_2602_18560_amd.profile_summary import kernel_source_hash
    if js.get("kernel") != kernel or js.get("source_sha256") != kernel_source_hash():
        return None
    return float(js["traffic_bytes_per_launch"])


def cpu_baseline(cat, run, iters=3):
    """The FP64 oracle on the same catalog, first `iters` loop bodies only."""
    from oracle import oracle as O
    threads = O.set_threads(all_threads())
    cfg = O.make_config(run, max_iter=iters)
    t0 = time.perf_counter()
    r = O.run(cat, cfg, spectra=False)
    dt = time.perf_counter() - t0
    done = r.n_iter
    return {"value": cat.n * done / dt, "unit": "binary-iterations/s", "cores": threads,
            "kind": "oracle", "host_cpu": host_cpu()["model"],
            "sample": f"the same {cat.n}-source catalog, first {done} loop bodies "
                      f"(prep + {done} x [binning, running median over all bins, SNR]), "
                      f"{dt:.1f} s on {threads} threads"}


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count()}


def all_threads():
    """OpenMP threads for an all-core leg: OMP_NUM_THREADS if set, else the
    cores this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    return int(env) if env.isdigit() and int(env) > 0 else len(os.sched_getaffinity(0))


def oracle_leg(cat, run, threads=0, max_iter=0):
    """Time the oracle on one catalog: `threads` OpenMP threads (0 = all),
    at most `max_iter` loop bodies (0 = the whole run)."""
    from oracle import oracle as O
    used = O.set_threads(threads if threads > 0 else all_threads())
    cfg = O.make_config(run, max_iter=max_iter)
    t0 = time.perf_counter()
    r = O.run(cat, cfg, spectra=False)
    dt = time.perf_counter() - t0
    if r.status not in (0, -6):
        raise RuntimeError(f"oracle run failed with status {r.status}")
    return {"n": int(cat.n), "threads": used, "bodies": int(r.n_iter), "complete": r.status == 0,
            "seconds": dt, "binary_iterations_per_s": cat.n * r.n_iter / dt}


def bench_oracle(args):
    """The FP64 oracle alone on the host cores: one thread on the 1e4 and 1e7
    catalogs, all threads on the 1e7 catalog, and all threads on a subset of
    the 64-catalog batch (the 8 smallest and the 2 largest, first loop bodies
    only), extrapolated to whole runs with the loop-body counts the GPU finds
    on the same catalogs."""
    from paper_2602_18560_amd.inputs import batch_populations, catalog_1e4, catalog_1e7, draw_catalog
    legs = {}
    cat, run = catalog_1e4()
    log("[oracle] 1e4 catalog, one thread, whole run")
    legs["1e4_single_thread"] = oracle_leg(cat, run, threads=1)
    log("[oracle] drawing the 1e7 catalog")
    cat, run = catalog_1e7(args.n)
    log(f"[oracle] 1e7 catalog, one thread, first {args.oracle_bodies_single} loop bodies")
    legs["1e7_single_thread"] = oracle_leg(cat, run, threads=1, max_iter=args.oracle_bodies_single)
    log(f"[oracle] 1e7 catalog, all threads, first {args.cpu_iters} loop bodies")
    legs["1e7_all_threads"] = oracle_leg(cat, run, threads=0, max_iter=args.cpu_iters)
    del cat
    pops, brun = batch_populations(args.catalogs)
    order = sorted(range(len(pops)), key=lambda j: pops[j].n)
    subset = order[:8] + order[-2:]
    bodies = args.oracle_bodies_batch
    sub = []
    n_iter_gpu = {}
    import torch
    ctx = None
    if torch.cuda.is_available():
        from paper_2602_18560_amd import gbsub as G
        torch.cuda.set_device(0)
        ctx = G.Context(G.config_from_run(brun))
    for j in subset:
        c = draw_catalog(pops[j])
        log(f"[oracle] batch catalog {j} (N = {c.n}), all threads, first {bodies} loop bodies")
        leg = oracle_leg(c, brun, threads=0, max_iter=bodies)
        leg["catalog"] = j
        if ctx is not None:
            n_iter_gpu[j] = int(ctx.run(G.DeviceCatalog.from_host(c)).n_iter)
            leg["n_iter"] = n_iter_gpu[j]
        sub.append(leg)
        del c
    work = sum(l["n"] * l["bodies"] for l in sub)
    secs = sum(l["seconds"] for l in sub)
    rate = work / secs
    batch = {"subset": subset, "legs": sub, "binary_iterations_per_s": rate, "seconds": secs}
    if n_iter_gpu:
        full_sub = sum(pops[j].n * n_iter_gpu[j] for j in subset)
        mean_iter = full_sub / sum(pops[j].n for j in subset)
        total = sum(p.n for p in pops)
        batch["extrapolated"] = {
            "subset_whole_runs_s": full_sub / rate,
            "all_catalogs_s": total * mean_iter / rate,
            "how": "measured rate on the subset's first loop bodies; whole runs take the GPU's "
                   "loop-body counts on the same catalogs; the 64 catalogs take the subset's "
                   "source-weighted mean count (an extrapolation, not a measurement)"}
    out = {"metric": "oracle binary-iterations/s", "unit": "binary-iterations/s",
           "host": host_cpu(), "legs": legs, "batch": batch,
           "config": {"workload": "FP64 oracle on the host cores: 1e4 catalog (seed 0, T = 1 yr, "
                                  "W = 251), 1e7 catalog (seed 2, T = 4 yr, W = 1001), and 10 of "
                                  "the 64 batch catalogs (meta seed 3)"}}
    print(json.dumps(out), flush=True)


def percentile(x, q):
    import numpy as np
    return float(np.percentile(np.asarray(x, dtype=np.float64), q))


def bench_batch(args):
    """Batched against plain on the same device-resident catalogs."""
    from paper_2602_18560_amd.inputs import batch_populations, draw_catalogs
    pops, run = batch_populations(args.catalogs)
    log(f"[batch] drawing {len(pops)} catalogs, {sum(p.n for p in pops):.3e} sources")
    t0 = time.perf_counter()
    cats = draw_catalogs(pops)
    log(f"[batch] drawn in {time.perf_counter() - t0:.1f} s")
    import torch
    from paper_2602_18560_amd import gbsub as G
    torch.cuda.set_device(0)
    dcs = [G.DeviceCatalog.from_host(c) for c in cats]
    schedule, table = {"tile_bins": 0, "split_blocks": 0}, []
    if not args.no_tune_batch:
        # one grid class here: the tuner times the whole batch per setting
        from paper_2602_18560_amd.autotune import tune_batch
        log("[batch] tuning the batch schedule (tile size, shared split budget)")
        schedule, table = tune_batch(dcs, [run] * len(dcs), chunk=args.chunk, log=log)
        log(f"[batch] schedule {schedule}")
    # plain runs keep the library's default schedule (the single-catalog one)
    pctxs = [G.Context(G.config_from_run(run)) for _ in cats]
    ctxs = [G.Context(G.config_from_run(run, **schedule)) for _ in cats]
    for c, d in zip(ctxs, dcs):
        c.ensure_workspace(d.n)
    for c, cb in zip(pctxs, ctxs):
        c.workspace = cb.workspace               # one workspace per catalog, used in turn
    torch.cuda.synchronize()
    n_tot = sum(d.n for d in dcs)

    def plain():
        out = [c.run(d) for c, d in zip(pctxs, dcs)]
        torch.cuda.synchronize()
        return out

    stream = torch.cuda.Stream()
    batch = G.Batch(len(dcs))

    def batched():
        for c, d in zip(ctxs, dcs):
            batch.admit(c, d, stream=stream)
        while True:
            state, running = batch.poll(stream)
            if running == 0:
                break
            batch.step(args.chunk, stream)
        out = []
        for k in range(len(dcs)):
            st, s = batch.retire(k, stream)
            if st != G.OK:
                raise G.GbsubError(st, "batched run")
            out.append(s)
        torch.cuda.synchronize()
        return out

    log("[batch] warmup")
    plain()
    batched()
    log("[batch] timed")
    tp, tb = [], []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        sp = plain()
        tp.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        sb = batched()
        tb.append(time.perf_counter() - t0)
    for a, b in zip(sp, sb):
        assert (a.n_iter, a.n_resolved, a.n_candidates) == (b.n_iter, b.n_resolved, b.n_candidates)
    bi = sum(d.n * s.n_iter for d, s in zip(dcs, sb))
    wb, wp = min(tb), min(tp)
    out = {
        "metric": "catalogs/h", "value": len(dcs) / wb * 3600.0, "unit": "catalogs/h", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": wb * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{len(dcs)} catalogs, N log-uniform in [1e5, 2e7] (meta seed 3, "
                               "catalog j seed 3000+j), per-catalog hyperparameters, T = 4 yr, "
                               "W = 1001, one shared batch, graph-captured loop bodies; catalogs "
                               "resident in HBM",
                   "n_catalogs": len(dcs), "n_sources": n_tot, "chunk": args.chunk,
                   "n_iter": [s.n_iter for s in sb], "batch_schedule": schedule,
                   "tuner_table_ms": [(t, sp, ms * 1e3) for t, sp, ms in table]},
        "plain": {"catalogs_per_h": len(dcs) / wp * 3600.0, "ms": wp * 1e3},
        "speedup_vs_plain": wp / wb,
        "binary_iterations_per_s": {"batched": bi / wb, "plain": bi / wp},
    }
    batch.close()
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Continuous batching of a Poisson job stream (saturated run first).
    Host catalogs: a pool of distinct catalogs drawn ahead into pinned host
    memory, job j running catalog j mod pool with its own T and W (every job
    still copies its catalog host-to-device at admission).  With --gpu-gen
    the jobs' catalogs come from the population model and are drawn on the GPU
    at admission (inside the latency; no host catalog).  Schedules are tuned
    per grid class on batches of pool catalogs; a sample of served jobs is
    re-run alone through gbsub_run and compared bit for bit."""
    import dataclasses
    import numpy as np
    if args.gpu_gen:
        from paper_2602_18560_amd.inputs import model_job_stream
        jobs = model_job_stream(args.jobs, rate_hz=1.0)
        log(f"[serve] {len(jobs)} model jobs, {sum(j.n for j in jobs):.3e} sources drawn on the GPU")
    else:
        from paper_2602_18560_amd.inputs import job_stream, draw_catalogs
        jobs = job_stream(args.jobs, rate_hz=1.0)
        npool = min(args.pool, len(jobs))
        log(f"[serve] drawing a pool of {npool} catalogs, "
            f"{sum(j.population.n for j in jobs[:npool]):.3e} sources")
        t0 = time.perf_counter()
        cats = draw_catalogs([j.population for j in jobs[:npool]])
        log(f"[serve] drawn in {time.perf_counter() - t0:.1f} s")
    import torch
    from paper_2602_18560_amd import gbsub as G
    from paper_2602_18560_amd import serve as SV
    from paper_2602_18560_amd.autotune import grid_class, tune_batch
    torch.cuda.set_device(0)
    schedules = {}
    if not args.gpu_gen:
        pinned = [SV.pin_catalog(c) for c in cats]
        if not args.no_tune_batch:
            classes = {}
            for j in jobs[:npool]:
                classes.setdefault(grid_class(j.run), []).append(j.index)
            for key, idx in classes.items():
                idx = sorted(idx, key=lambda i: cats[i].n)[-8:]          # the 8 largest of the class
                dcs = [G.DeviceCatalog.from_host(cats[i]) for i in idx]
                log(f"[serve] tuning grid class T = {key[0] / 31557600:.0f} yr on {len(idx)} catalogs")
                schedules[key], _ = tune_batch(dcs, [jobs[i].run for i in idx], chunk=args.chunk)
                log(f"[serve]   schedule {schedules[key]}")
                del dcs
                torch.cuda.empty_cache()
        del cats

    def requests(times):
        if args.gpu_gen:
            return [SV.model_request(dataclasses.replace(j, arrival_s=t)) for j, t in zip(jobs, times)]
        return [SV.Request(j.index, t, *pinned[j.index % npool], run=j.run) for j, t in zip(jobs, times)]

    budget = args.budget_gb * 2**30
    log("[serve] warmup")
    SV.serve(requests([0.0] * min(4, len(jobs)))[:4], args.slots, budget, args.chunk, schedules=schedules)
    log(f"[serve] saturated run (every job queued at t = 0), {len(jobs)} jobs")
    prog = lambda k, n: log(f"[serve]   {k} / {n} jobs done")
    done, srv = SV.serve(requests([0.0] * len(jobs)), args.slots, budget, args.chunk, schedules=schedules,
                         progress=prog)
    makespan = max(c.done_s for c in done)
    cap = len(done) / makespan
    rate = args.load * cap
    log(f"[serve] capacity {cap:.2f} jobs/s; Poisson run at {rate:.2f} jobs/s")
    times = [j.arrival_s / rate for j in jobs]          # unit-rate arrivals, rescaled
    # a sample of jobs whose served results are kept: the smallest ones of
    # each grid class and the largest job
    by_n = sorted(range(len(jobs)), key=lambda i: (jobs[i].n if args.gpu_gen else jobs[i % npool].population.n))
    check = set(by_n[:max(args.check_jobs - 1, 0)] + by_n[-1:]) if args.check_jobs else set()
    done2, srv2 = SV.serve(requests(times), args.slots, budget, args.chunk, schedules=schedules,
                           keep_jobs=check, progress=prog)
    bad = [c for c in done + done2 if c.status != 0]
    if bad:
        raise RuntimeError(f"{len(bad)} jobs did not settle")
    # served == alone, bit for bit, on the sample
    checked = []
    reqs = {r.index: r for r in requests(times)}
    for c in done2:
        if c.context is None:
            continue
        r = reqs[c.index]
        ctx = G.Context(G.config_from_run(r.run, **schedules.get(grid_class(r.run), {})))
        if args.gpu_gen:
            dc = G.generate(r.model, r.seed, r.n)
        else:
            dc = G.DeviceCatalog(*(x.to("cuda") for x in (r.A, r.f, r.fdot, r.ids)))
        s = ctx.run(dc)
        same = (s.n_iter == c.summary.n_iter and s.n_resolved == c.summary.n_resolved
                and np.array_equal(ctx.spectrum(G.SPEC_SN), c.context.spectrum(G.SPEC_SN))
                and all(np.array_equal(a, b) for a, b in zip(ctx.resolved(), c.context.resolved())))
        checked.append({"job": c.index, "n": c.n_sources, "t_obs_yr": round(r.run.t_obs_s / 31557600),
                        "n_iter": s.n_iter, "equal_alone": bool(same)})
        ctx.close()
        c.context.close()
    if not all(x["equal_alone"] for x in checked):
        raise RuntimeError(f"served results differ from runs alone: {checked}")
    lat = [c.latency_s for c in done2]
    span2 = max(c.done_s for c in done2) - min(c.arrival_s for c in done2)
    hb, hms = srv2.h2d_stats()
    bi = sum(c.n_sources * c.summary.n_iter for c in done2)
    out = {
        "metric": "p99 latency", "value": percentile(lat, 99) * 1e3, "unit": "ms", "n_gpus": 1,
        "steps": len(jobs), "warmup": 4, "ms_per_step": span2 / len(jobs) * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"{len(jobs)} jobs, Poisson arrivals at {args.load}x the saturated "
                                "rate, T in {1,2,4} yr with W = 251/501/1001 " + (
                                    "(meta seed 7, job j generator seed 7000+j); catalogs of N "
                                    "log-uniform in [1e5, 3e7] drawn on the GPU from the population "
                                    "model at admission, hyperparameters uniform in the prior box, "
                                    "generation inside the latency"
                                    if args.gpu_gen else
                                    f"(meta seed 5); job j runs catalog j mod {npool} of a pool drawn "
                                    "ahead into pinned host memory (pool catalog i: the job stream's "
                                    "population i, N log-uniform in [1e5, 3e7], seed 5000+i); H2D "
                                    "inside the latency")),
                   "slots": args.slots, "budget_gb": args.budget_gb, "chunk": args.chunk,
                   "schedules": {f"{k[0] / 31557600:.0f}yr_W{k[3]}": v for k, v in schedules.items()}},
        "latency_ms": {"p50": percentile(lat, 50) * 1e3, "p99": percentile(lat, 99) * 1e3,
                       "max": max(lat) * 1e3},
        "throughput_jobs_per_s": len(done2) / span2,
        "catalogs_per_h": len(done2) / span2 * 3600.0,
        "saturated_jobs_per_s": cap,
        "binary_iterations_per_s": bi / span2,
        "h2d": {"GB": hb / 1e9, "ms": hms, "GBps": hb / 1e9 / (hms * 1e-3) if hms else None},
        "served_equal_alone": checked,
    }
    print(json.dumps(out), flush=True)


def bench_generate(args):
    """Catalogs drawn on the GPU from the population model (gbsub_generate):
    generator throughput, then generation + subtraction of one catalog."""
    import torch
    from paper_2602_18560_amd import gbsub as G
    from paper_2602_18560_amd.inputs import RunConfig, YEAR_S
    torch.cuda.set_device(0)
    n = int(args.n) if args.n != 10_000_000 else 7_500_000      # N_b of the paper's figure
    pop = G.population(**G.PAPER_FIG_LAMBDA)
    dc = G.generate(pop, 1, n)
    torch.cuda.synchronize()
    log(f"[generate] {n} sources x{args.steps}")
    t0 = time.perf_counter()
    for s in range(args.steps):
        G.generate(pop, 100 + s, n, out=dc)
    torch.cuda.synchronize()
    gen_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    run = RunConfig(t_obs_s=4 * YEAR_S, f_min_hz=1e-4, f_max_hz=1e-2, window_bins=1001)
    ctx = G.Context(G.config_from_run(run))
    ctx.ensure_workspace(n)
    G.generate(pop, 7, n, out=dc)
    s = ctx.run(dc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        G.generate(pop, 7, n, out=dc)
        s = ctx.run(dc)
    torch.cuda.synchronize()
    e2e_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ctx.close()
    out = {"metric": "sources/s", "value": n / (gen_ms * 1e-3), "unit": "sources/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 1, "ms_per_step": gen_ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{n} sources drawn on the GPU from the population model with the "
                                  "hyperparameters of the paper's population-model figure "
                                  "(alpha_PL -2.9, alpha_G 1.96, beta_G 1.8, mu_G -21, mu -22, "
                                  "sigma 0.18, rho 0.99) on [0.1, 10] mHz",
                      "n_sources": n},
           "generate_and_subtract": {"ms": e2e_ms, "t_obs_yr": 4, "window_bins": 1001,
                                     "n_iter": s.n_iter, "n_resolved": s.n_resolved,
                                     "n_candidates": s.n_candidates}}
    print(json.dumps(out), flush=True)


def bench_precision(args):
    """FP64 / FP32 compensated / naive FP32 against the oracle (tests/golden)."""
    import numpy as np
    import torch
    from paper_2602_18560_amd import gbsub as G
    from paper_2602_18560_amd.inputs import catalog_1e7
    gold = np.load(os.path.join(ROOT, "tests", "golden", "catalog1e7_oracle.npz"))
    grho = np.load(os.path.join(ROOT, "tests", "golden", "catalog1e7_rho2.npz"))
    log("[precision] drawing the 1e7-binary catalog")
    cat, run = catalog_1e7()
    torch.cuda.set_device(0)
    dc = G.DeviceCatalog.from_host(cat)
    ref_ids = gold["resolved_ids"].astype(np.int64)
    ref_it = gold["resolved_iter"]
    bins = gold["S_bins"]
    S_ref, X_ref = gold["S_final"], gold["X_final"]
    out_modes = {}
    for name, prec in (("fp64", G.FP64), ("fp32_compensated", G.FP32_COMP), ("fp32_naive", G.FP32_NAIVE)):
        ctx = G.Context(G.config_from_run(run, precision=prec))
        ctx.ensure_workspace(cat.n)
        s = ctx.run(dc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            s = ctx.run(dc)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        S = ctx.spectrum(G.SPEC_SN)[bins]
        X = ctx.spectrum(G.SPEC_X_RESIDUAL)[bins]
        ids, it = ctx.resolved()
        cids, cit, cr2 = ctx.candidates()
        ctx.close()
        relS = np.abs(S - S_ref) / S_ref
        xo = X_ref
        pos = xo > 0
        relX = np.abs(X[pos] - xo[pos]) / xo[pos]
        relXS = np.abs(X - xo) / S_ref          # X error on the scale of the PSD it enters
        same = np.array_equal(cids.astype(np.int64), grho["cand"].astype(np.int64))
        relR = np.abs(cr2 - grho["rho2"]) / grho["rho2"] if same else np.array([np.nan])
        a = set(ref_ids.tolist())
        b = set(ids.astype(np.int64).tolist())
        both = np.intersect1d(ref_ids, ids.astype(np.int64))
        it_ref = dict(zip(ref_ids.tolist(), ref_it.tolist()))
        it_gpu = dict(zip(ids.astype(np.int64).tolist(), it.tolist()))
        moved = int(sum(it_ref[i] != it_gpu[i] for i in both.tolist()))
        out_modes[name] = {
            "ms_per_step": ms, "n_iter": s.n_iter, "n_iter_oracle": int(gold["n_iter"]),
            "n_resolved": s.n_resolved, "n_candidates": s.n_candidates,
            "flips_resolved_only_gpu": len(b - a), "flips_resolved_only_oracle": len(a - b),
            "same_set_other_iteration": moved,
            "S_rel_err": {"max": float(relS.max()), "median": float(np.median(relS)),
                          "bins": int(relS.size)},
            "X_rel_err": {"max": float(relX.max()), "median": float(np.median(relX)),
                          "bins": int(relX.size),
                          "nonzero_where_oracle_zero": int(np.count_nonzero(X[~pos])),
                          "max_abs_err_over_S": float(relXS.max())},
            "rho2_rel_err": {"max": float(np.nanmax(relR)), "median": float(np.nanmedian(relR)),
                             "candidates": int(relR.size)},
        }
        log(f"[precision] {name}: {out_modes[name]}")
    out = {"metric": "resolve-decision flips vs FP64 oracle (FP32 compensated)",
           "value": out_modes["fp32_compensated"]["flips_resolved_only_gpu"]
           + out_modes["fp32_compensated"]["flips_resolved_only_oracle"],
           "unit": "sources", "n_gpus": 1, "steps": args.steps, "warmup": 1,
           "ms_per_step": out_modes["fp32_compensated"]["ms_per_step"], "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "1e7-binary catalog (seed 2), T = 4 yr, W = 1001, in FP64 / "
                                  "FP32 with double-fp32 (compensated) sums / naive FP32; S and X "
                                  "on every 997th bin, rho^2 of every candidate at its last "
                                  "evaluation, resolved ids and loop bodies against the FP64 "
                                  "oracle's stored results (every bin: tests/test_gpu_precision.py)"},
           "modes": out_modes}
    print(json.dumps(out), flush=True)


# Algorithmic work per unit of the complex-template model's kernel families.
# HBM-bound: bytes per unit.  Template-bound (FFT synthesis of a 128-sample
# template in fp64): counted flops per template -- the 128-point complex FFT
# 5 N log2 N = 4480, the sample phases and scaling 128 x 8 = 1024, the
# power-weighted sum 128 x 5 = 640; the evaluations of exp(2 pi i t) per
# sample are not counted.
CX_ALGO = {
    "xupdate": ("hbm", 48.0),        # per bin: read 4 int64 of h, write X_A, X_E
    "median": ("hbm", 24.0),         # per output bin and channel: read X and S_instr, write S
    "prep": ("alu", 6144.0),         # per source: one template (injection and candidate cut)
    "snr": ("alu", 6144.0),          # per candidate evaluation: one template
}
FP64_VECTOR_PEAK_TFLOPS = 78.6


def bench_cx(args):
    """The complex-template data model (gbsub_cx_run) on the 1e7 catalog with
    its channel phases: whole runs, inputs resident in HBM."""
    import numpy as np
    import torch
    from paper_2602_18560_amd import gbsub as G
    from paper_2602_18560_amd.inputs import catalog_cx_1e7
    log("[cx] drawing the 1e7-binary catalog and its template phases")
    cat, pa, pe, run = catalog_cx_1e7()
    if args.n != 10_000_000:
        sub = np.arange(int(args.n))
        cat, pa, pe = cat.subset(sub), pa[sub], pe[sub]
    torch.cuda.set_device(0)
    dc = G.DeviceCxCatalog.from_host(cat, pa, pe)
    ctx = G.Context(G.config_from_run(run))
    cx = G.CxRun(ctx)
    cx.ensure_workspace(cat.n)
    for _ in range(max(args.warmup, 1)):
        s = cx.run(dc)
    torch.cuda.synchronize()
    log(f"[cx] n_iter={s.n_iter} candidates={s.n_candidates} resolved={s.n_resolved}; timing {args.steps} runs")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s = cx.run(dc)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # one more run with HIP events around every kernel family
    ctx.set_profiling(True)
    cx.run(dc)
    torch.cuda.synchronize()
    stats = ctx.kernel_stats()
    ctx.set_profiling(False)
    ctx.close()
    fams = {}
    for name, st in stats.items():
        if name not in CX_ALGO or st["launches"] == 0:
            continue
        bound, per = CX_ALGO[name]
        avg_ms = st["total_ms"] / st["launches"]
        units = st["units"] / st["launches"]
        if bound == "hbm":
            ach, peak, unit = per * units / (avg_ms * 1e-3) / 1e9, 8000.0, "GB/s"
        else:
            ach, peak, unit = per * units / (avg_ms * 1e-3) / 1e12, FP64_VECTOR_PEAK_TFLOPS, "TFLOP/s"
        fams[name] = {"launches": st["launches"], "total_ms": st["total_ms"], "avg_launch_ms": avg_ms,
                      "units_per_launch": units, "bound": bound, "achieved": ach, "peak": peak, "unit": unit,
                      "frac": ach / peak}
    dom = max(fams, key=lambda k: fams[k]["total_ms"])
    d = fams[dom]
    roof = {"bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"], "unit": d["unit"],
            "frac": d["frac"], "traffic": None, "kernel": dom, "avg_launch_ms": d["avg_launch_ms"]}
    out = {"metric": "binary-iterations/s", "value": cat.n * s.n_iter / (ms * 1e-3),
           "unit": "binary-iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": max(args.warmup, 1),
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"complex-template data model: {cat.n}-binary catalog (seed 2, phases "
                                  "seed 2), T = 4 yr, [0.1, 30] mHz (3,774,290 bins), 128-sample templates "
                                  "in A and E, running median W = 1001 per channel, rho_th = 7",
                      "n_iter": s.n_iter, "n_candidates": s.n_candidates, "n_resolved": s.n_resolved},
           "roofline": roof, "families": fams}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cx_cpu_baseline(cat, pa, pe, run)
    print(json.dumps(out), flush=True)


def cx_cpu_baseline(cat, pa, pe, run, n_sub=100_000):
    """The complex-template oracle on the first n_sub sources of the same
    catalog and grid, one loop body."""
    from oracle import oracle as O
    threads = O.set_threads(all_threads())
    sub = slice(0, min(n_sub, cat.n))
    from paper_2602_18560_amd.inputs import Catalog
    c2 = Catalog(cat.A[sub], cat.f[sub], cat.fdot[sub], cat.id[sub])
    cfg = O.make_config(run, max_iter=1)
    t0 = time.perf_counter()
    r = O.cx_run(c2, pa[sub], pe[sub], cfg, spectra=False)
    dt = time.perf_counter() - t0
    return {"value": c2.n * r.n_iter / dt, "unit": "binary-iterations/s", "cores": threads, "kind": "oracle",
            "host_cpu": host_cpu()["model"],
            "sample": f"the first {c2.n} sources of the same catalog on the same grid, {r.n_iter} loop body "
                      f"(templates, injection, candidate cut, per-channel running median over all bins, SNR), "
                      f"{dt:.1f} s on {threads} threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["1e7", "batch", "serve", "precision", "generate", "oracle", "cx"],
                    default="1e7")
    ap.add_argument("--catalogs", type=int, default=64, help="batch: number of catalogs")
    ap.add_argument("--jobs", type=int, default=2000, help="serve: number of jobs")
    ap.add_argument("--slots", type=int, default=64, help="serve: batch slots")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serve: device memory budget")
    ap.add_argument("--load", type=float, default=0.7, help="serve: arrival rate / saturated rate")
    ap.add_argument("--chunk", type=int, default=4, help="loop bodies per batch step")
    ap.add_argument("--no-tune-batch", action="store_true",
                    help="batch / serve: the default schedule instead of the batch tuner's per grid class")
    ap.add_argument("--pool", type=int, default=64,
                    help="serve: distinct catalogs drawn on the host; job j runs catalog j mod pool")
    ap.add_argument("--check-jobs", type=int, default=4,
                    help="serve: served jobs re-run alone through gbsub_run and compared bit for bit")
    ap.add_argument("--gpu-gen", action="store_true",
                    help="serve: catalogs drawn on the GPU from the population model at admission")
    ap.add_argument("--estimator", choices=["median", "mean"], default="median",
                    help="1e7 workload: running median (default) or running mean")
    ap.add_argument("--window", type=int, default=0, help="1e7 workload: window bins (default 1001)")
    ap.add_argument("--tune", action="store_true",
                    help="1e7 workload: run the schedule tuner first (default: the library's default "
                         "schedule, tile 2048 and split budget 512, the one the committed profiles use)")
    ap.add_argument("--no-tune", action="store_true", help="(the default; kept for old command lines)")
    ap.add_argument("--schedule", default="",
                    help="1e7 workload: TILE,SPLIT fixed schedule (tile bins, split budget), no tuning")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=10_000_000, help="catalog size (default: 1e7)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=9)
    ap.add_argument("--oracle-bodies-single", type=int, default=1,
                    help="oracle workload: loop bodies of the one-thread 1e7 run")
    ap.add_argument("--oracle-bodies-batch", type=int, default=2,
                    help="oracle workload: loop bodies per batch catalog")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); catalogs are independent "
              "and shard across GPUs with no communication, see DESIGN.md", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "precision":
        return bench_precision(args)
    if args.workload == "generate":
        return bench_generate(args)
    if args.workload == "oracle":
        return bench_oracle(args)
    if args.workload == "cx":
        return bench_cx(args)

    import numpy as np
    import torch

    from paper_2602_18560_amd import gbsub as G
    from paper_2602_18560_amd.inputs import catalog_1e7

    log("[bench] drawing the 1e7-binary catalog")
    cat, run = catalog_1e7(args.n)
    overrides = {"estimator": G.MEAN if args.estimator == "mean" else G.MEDIAN}
    if args.window:
        overrides["window_bins"] = args.window
    torch.cuda.set_device(0)
    dc = G.DeviceCatalog.from_host(cat)
    schedule = {"tile_bins": 0, "split_blocks": 0}
    if args.schedule:
        tile, split = (int(v) for v in args.schedule.split(","))
        schedule = {"tile_bins": tile, "split_blocks": split}
    elif args.tune:
        from paper_2602_18560_amd.autotune import tune
        log("[bench] tuning the schedule (tile size, split budget)")
        schedule, _ = tune(dc, {**run.as_dict(), **overrides}, log=log)
        log(f"[bench] schedule {schedule}")
    ctx = G.Context(G.config_from_run(run, **overrides, **schedule))
    ctx.ensure_workspace(cat.n)
    torch.cuda.synchronize()

    log(f"[bench] warmup x{args.warmup}")
    for _ in range(args.warmup):
        s = ctx.run(dc)
    torch.cuda.synchronize()

    # Whole-run throughput: K runs with no events anywhere (an event on a
    # dispatch leaves the GPU idle for a few microseconds on each side).
    fam = "median"
    log(f"[bench] timed x{args.steps}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s = ctx.run(dc)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    value = cat.n * s.n_iter / (ms * 1e-3)
    # The dominant kernel's launch durations: the same K runs again, with
    # HIP events carried by every working median dispatch (on its stream).
    log(f"[bench] median launch durations (HIP events) x{args.steps}")
    ctx.set_profiling(1 << G.KF_MEDIAN)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        ctx.run(dc)
    torch.cuda.synchronize()
    ms_ev = (time.perf_counter() - t2) * 1e3 / args.steps
    st = ctx.kernel_stats()[fam]
    avg_ms = st["total_ms"] / max(st["launches"], 1)
    bytes_per_launch = ALGO_BYTES[fam] * st["units"] / max(st["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9

    # The first body filters every bin (full grid); later bodies only the
    # tiles a subtraction touched.  The first launch alone: runs stopped
    # after one body (max_iter = 1), median events only.
    ctx1 = G.Context(G.config_from_run(run, **overrides, **schedule, max_iter=1))
    ctx1.ensure_workspace(cat.n)
    ctx1.set_profiling(1 << G.KF_MEDIAN)
    for _ in range(args.steps):
        st1, _ = ctx1.run_raw(dc)
        if st1 not in (G.OK, G.E_MAXITER):
            raise G.GbsubError(st1, "gbsub_run (first body)")
    torch.cuda.synchronize()
    st_first = ctx1.kernel_stats()[fam]
    ctx1.close()
    first_ms = st_first["total_ms"] / max(st_first["launches"], 1)
    first_units = st_first["units"] / max(st_first["launches"], 1)
    late_launches = st["launches"] - st_first["launches"]
    late_ms = (st["total_ms"] - st_first["total_ms"]) / max(late_launches, 1)
    late_units = (st["units"] - st_first["units"]) / max(late_launches, 1)
    launch_split = {
        "first_body": {"avg_launch_ms": first_ms, "bins_per_launch": first_units,
                       "achieved_GBs": ALGO_BYTES[fam] * first_units / (first_ms * 1e-3) / 1e9},
        "later_bodies": {"avg_launch_ms": late_ms, "bins_per_launch": late_units,
                         "achieved_GBs": ALGO_BYTES[fam] * late_units / (late_ms * 1e-3) / 1e9},
    }

    nprof = min(args.steps, 5)
    log(f"[bench] per-family breakdown (profiled, untimed) x{nprof}")
    ctx.set_profiling(True)
    for _ in range(nprof):
        ctx.run(dc)
    torch.cuda.synchronize()
    stats = ctx.kernel_stats()
    ctx.set_profiling(False)
    kern = {k: {"ms_per_step": round(v["total_ms"] / nprof, 4),
                "launches_per_step": v["launches"] / nprof,
                "units_per_step": v["units"] / nprof, "unit": v["unit"]}
            for k, v in stats.items() if v["launches"]}
    total_algo = sum(ALGO_BYTES[k] * stats[k]["units"] for k in ALGO_BYTES) / nprof
    out = {
        "metric": "binary-iterations/s",
        "value": value,
        "unit": "binary-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"1e7-binary catalog (seed 2), f in [0.1, 30] mHz, T_obs = 4 yr, "
                               f"3,774,290 bins of 1/T, running-{args.estimator} window "
                               f"{args.window or 1001}, rho_th = 7; catalog resident in HBM",
                   "n_sources": cat.n, "n_bins": s.n_bins, "n_iter": s.n_iter,
                   "n_candidates": s.n_candidates, "n_resolved": s.n_resolved,
                   "schedule": schedule},
        "roofline": {"bound": "hbm", "kernel": "k_" + args.estimator, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("k_median") if args.estimator == "median" else None,
                     "avg_launch_ms": avg_ms, "algo_bytes_per_launch": bytes_per_launch,
                     "launches": st["launches"], "ms_per_step_with_events": ms_ev,
                     "bytes_per_bin": ALGO_BYTES[fam], "launch_split": launch_split},
        "run_level_hbm": {"algo_bytes_per_step": total_algo,
                          "achieved_GBs": total_algo / (ms * 1e-3) / 1e9,
                          "frac": total_algo / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "kernels": kern,
    }
    if not args.no_cpu_baseline:
        log(f"[bench] oracle sample: first {args.cpu_iters} loop bodies on the host cores")
        out["cpu_baseline"] = cpu_baseline(cat, run, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
