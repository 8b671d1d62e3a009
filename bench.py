"""Benchmark: prime implicants of one n = 24 function on one MI355X.

One step = the whole hot path on one resident truth table: implicants
(MergeAll), primes (ReduceAll), the prime bitmap and the sorted prime list
written to HBM (dqmc_primes).  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
PAPER_N24_SECONDS = 120.0  # Table 1, DenseQMC at n = 24 (one EPYC core), context only


def csrc_hash() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2302_10083_amd", "csrc")
    for fn in sorted(os.listdir(d)):
        with open(os.path.join(d, fn), "rb") as f:
            h.update(fn.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, workload: str):
    """HBM traffic measured with rocprofv3 counters for this kernel source, from
    profiles/pmc_<kernel>_<workload>.md (lines 'key: value'); None when absent
    or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip().lstrip("- ")] = v.strip()
    if kv.get("csrc_hash") != csrc_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def host_info():
    """nproc, CPU model and RAM of the host the baseline ran on."""
    info = {"nproc": os.cpu_count(), "cpu_share": len(os.sched_getaffinity(0))}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["ram_GB"] = round(int(line.split()[1]) * 1024 / 1e9, 1)
                    break
    except OSError:
        pass
    return info


def baseline_threads(requested):
    """Host threads for the oracle: every core of this process's CPU share,
    at most 16 (one GPU's share of the host cores) unless asked otherwise."""
    if requested > 0:
        return requested
    return max(1, min(len(os.sched_getaffinity(0)), 16))


def oracle_o2_seconds(n, tt, threads):
    """The oracle's definitional enumerator (O2: the M sweep of the Lemma of
    Sec. 4.1, then the O formula over every cube), timed on the host."""
    import oracle

    t0 = time.perf_counter()
    M = oracle.enum_M(n, tt, threads)
    t1 = time.perf_counter()
    O = oracle.enum_O(n, M, threads)
    t2 = time.perf_counter()
    lst, cnt = oracle.extract(n, O)
    t3 = time.perf_counter()
    return dict(M_s=t1 - t0, O_s=t2 - t1, extract_s=t3 - t2, total_s=t3 - t0, primes=int(cnt)), lst


def cpu_baseline(n, tt, sub_n, threads):
    """O2 on a bounded sample of the workload: the restriction of f to
    x_(sub_n+1) = ... = x_n = 0, a function of sub_n variables whose cubes are
    the first 3^sub_n cubes of f's cube space (the block whose top n - sub_n
    digits are all 0).  Returns (cubes/s, threads, details, sorted primes of
    the restriction)."""
    import numpy as np

    sub_n = min(sub_n, n)
    words = max(1, (1 << sub_n) // 32)
    sub_tt = np.ascontiguousarray(np.asarray(tt, dtype=np.uint32)[:words])
    if sub_n < 5:
        sub_tt = sub_tt & np.uint32((1 << (1 << sub_n)) - 1)
    det, lst = oracle_o2_seconds(sub_n, sub_tt, threads)
    return 3**sub_n / det["total_s"], threads, det, sub_tt, lst


BATCH_WORKLOAD = "8192_n6_16"
SLOT_BYTES = 4 * 17504  # a tile of a state with n > 12 and its padding


def batch_model_bytes(ns, counts):
    """Algorithmic HBM bytes of one run of the batch launches, per job:
    n <= 12 (one workgroup): the truth table, the state and the list;
    13 <= n <= 16 (h = n - 12, 3^h tiles): the truth table, the 2^h binary
    tiles written and read back, every slot written by the column pass, every
    tile read and written by the final reduce, 40 B of summary per tile, the
    scan's 12 B per tile and the list.  The list pass's reads of non-zero
    chunks depend on the data and are not counted."""
    total = 0
    for n, c in zip(ns, counts):
        tt = 4 * max(1, 2 ** (n - 5)) if n >= 5 else 4
        if n <= 12:
            total += tt + 4 * 8 * 3 ** max(n - 5, 0) + 8 * c + 8
        else:
            h = n - 12
            total += (tt + 2 * 2**h * SLOT_BYTES + 3**h * SLOT_BYTES + 3**h * 2 * (SLOT_BYTES - 32)
                      + 3**h * (40 + 12) + 8 * c + 8)
    return total


def bench_batch(ctx, reps=5):
    """Batched workload (8192 functions, n uniform 6..16): the graph-replayed
    batch plan (a device-resident job array, planned on the device) against
    one dqmc_primes launch sequence per function."""
    import torch

    from paper_2302_10083_amd import dqmc, inputs

    specs = inputs.batch_specs(8192, seed=8192)
    dev = ctx.torch_device
    jobs = []
    for s in specs:
        n = s["n"]
        jobs.append(dict(n=n, tt=ctx.tt_to_device(inputs.make(s)), state=ctx.new_state(n), list=None, list_cap=0,
                         count=torch.zeros(1, dtype=torch.int64, device=dev)))
    dqmc.dqmc_primes_batch(ctx.ctx, jobs)  # count-only pass sizes the lists
    for j in jobs:
        c = int(j["count"].item())
        j["list"] = torch.empty(max(c, 1), dtype=torch.int64, device=dev)
        j["list_cap"] = c
    plan = dqmc.Batch(ctx.ctx, jobs)
    plan.run()
    torch.cuda.synchronize()
    trials = plan.autotune(reps=2)  # keeps the fastest column cap / item order on the plan
    best = min(trials, key=lambda t: t["ms"])
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            plan.run()
    torch.cuda.current_stream().wait_stream(st)
    g.replay()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        g.replay()
    b.record()
    torch.cuda.synchronize()
    ms_batch = a.elapsed_time(b) / reps
    # the enqueue-only call on the same device job table (no host knowledge of
    # the jobs' sizes: grids by bounds)
    dqmc.dqmc_primes_batch(ctx.ctx, plan.table, njobs=len(jobs))
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        dqmc.dqmc_primes_batch(ctx.ctx, plan.table, njobs=len(jobs))
    b.record()
    torch.cuda.synchronize()
    ms_call = a.elapsed_time(b) / reps
    # one launch sequence per function, same buffers
    for _ in range(2):
        for j in jobs:
            dqmc.dqmc_primes(ctx.ctx, j["n"], j["tt"], j["state"], j["list"], j["list_cap"], j["count"])
    torch.cuda.synchronize()
    a.record()
    for j in jobs:
        dqmc.dqmc_primes(ctx.ctx, j["n"], j["tt"], j["state"], j["list"], j["list_cap"], j["count"])
    b.record()
    torch.cuda.synchronize()
    ms_single = a.elapsed_time(b)
    state_bytes = sum(4 * dqmc.dqmc_state_words(s["n"]) for s in specs)
    model = batch_model_bytes([s["n"] for s in specs], [int(j["count"].item()) for j in jobs])
    traffic = read_traffic("batch", BATCH_WORKLOAD)
    del g
    plan.close()
    return {"workload": "8192 functions, n uniform 6..16, half Bernoulli half DNF (seed 8192)",
            "fns": len(specs), "state_GB": state_bytes / 1e9,
            "ms": ms_batch, "fns_per_s": len(specs) / (ms_batch / 1e3),
            "dqmc_primes_batch_call_ms": ms_call,
            "per_fn_launch_ms": ms_single, "per_fn_launch_fns_per_s": len(specs) / (ms_single / 1e3),
            "speedup_vs_per_fn_launch": ms_single / ms_batch, "graph_captured": True,
            # byte model of one run (batch_model_bytes) and, when profiles/
            # holds counters for these sources, the HBM bytes they measured
            "roofline": {"bound": "hbm", "model_GB": model / 1e9, "model_GBps": model / (ms_batch / 1e3) / 1e9,
                         "frac_model": model / (ms_batch / 1e3) / 1e9 / HBM_PEAK_GBPS,
                         "traffic_GB": traffic / 1e9 if traffic else None,
                         "traffic_GBps": traffic / (ms_batch / 1e3) / 1e9 if traffic else None,
                         "frac_traffic": traffic / (ms_batch / 1e3) / 1e9 / HBM_PEAK_GBPS if traffic else None},
            "autotune": {"col_cap": best["col_cap"], "order": best["order"],
                         "trials": [[t["col_cap"], t["order"], round(t["ms"], 3)] for t in trials]}}


def bench_sparse(ctx, n=24, densities=(0.25, 0.5), reps=3):
    """Sparse path (level-by-level QMC with hash sets) against the dense path
    on random functions of the paper's Table 1 densities."""
    import numpy as np
    import torch

    from paper_2302_10083_amd import dqmc, inputs

    dev = ctx.torch_device
    rows = []
    for d in densities:
        tt = inputs.bernoulli(n, d, 2400 + int(100 * d))
        ttd = ctx.tt_to_device(tt)
        count = torch.zeros(1, dtype=torch.int64, device=dev)
        # size the workspace from a first run's report
        work = torch.empty(8 << 30, dtype=torch.uint8, device=dev)
        rc, lv, npr = dqmc.dqmc_sparse_primes(ctx.ctx, n, ttd, None, 0, count, work)
        while rc != dqmc.DQMC_OK:
            del work
            torch.cuda.empty_cache()
            work = torch.empty(dqmc.dqmc_sparse_workspace_bytes(n, 2 * lv, 2 * max(npr, 1)), dtype=torch.uint8,
                               device=dev)
            rc, lv, npr = dqmc.dqmc_sparse_primes(ctx.ctx, n, ttd, None, 0, count, work)
        c = int(count.item())
        lst = torch.empty(max(c, 1), dtype=torch.int64, device=dev)
        dqmc.dqmc_sparse_primes(ctx.ctx, n, ttd, lst, c, count, work)
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            dqmc.dqmc_sparse_primes(ctx.ctx, n, ttd, lst, c, count, work)  # synchronous
            times.append(time.perf_counter() - t0)
        ms_sparse = 1e3 * min(times)
        sh = torch.zeros(1, dtype=torch.int64, device=dev)
        dqmc.dqmc_hash_words(ctx.ctx, lst, 2 * c, sh)
        del work
        torch.cuda.empty_cache()
        # the dense path on the same function
        state = ctx.new_state(n)
        dl = torch.empty(max(c, 1), dtype=torch.int64, device=dev)
        dqmc.dqmc_primes(ctx.ctx, n, ttd, state, dl, c, count)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            dqmc.dqmc_primes(ctx.ctx, n, ttd, state, dl, c, count)
        b.record()
        torch.cuda.synchronize()
        ms_dense = a.elapsed_time(b) / reps
        dh = torch.zeros(1, dtype=torch.int64, device=dev)
        dqmc.dqmc_hash_words(ctx.ctx, dl, 2 * c, dh)
        torch.cuda.synchronize()
        rows.append({"density": d, "primes": c, "largest_level": lv, "ms_sparse": ms_sparse, "ms_dense": ms_dense,
                     "same_list": int(sh.item()) == int(dh.item()) and int(count.item()) == c})
        del state, dl, lst
        torch.cuda.empty_cache()
    return {"workload": "n=%d Bernoulli(d) truth tables (seeds 2400+100d), the paper's Table 1 densities" % n,
            "rows": rows}


def bench_sliced(ctx, workload="c3x_n26_dnf2000_noise", ts=((2, 1), (2, 3), (1, 1)), reps=2):
    """Functions past one state in HBM: the sliced path on the n = 26 (or 27)
    version of the benchmark workload (two slice states of n - t variables)."""
    import numpy as np
    import torch

    from paper_2302_10083_amd import dqmc, inputs

    spec = inputs.CONFIGS[workload]
    n = spec["n"]
    tt = inputs.make(spec)
    dev = ctx.torch_device
    ttd = ctx.tt_to_device(tt)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    out = {"workload": workload, "n": n, "cubes": 3**n, "truth_table": spec,
           "single_state_GB": 4 * 17504 * 3 ** (n - 12) / 1e9, "rows": []}  # 3^(n-12) padded tile slots
    lst = None
    for t, nm in ts:
        need = (1 + nm) * 4 * dqmc.dqmc_state_words(n - t)
        try:
            o = ctx.new_state(n - t)
            m = [ctx.new_state(n - t) for _ in range(nm)]
            if lst is None:
                dqmc.dqmc_primes_sliced_multi(ctx.ctx, n, t, ttd, 0, o, m, None, 0, count)
                torch.cuda.synchronize()
                nprimes = int(count.item())
                lst = torch.empty(max(nprimes, 1), dtype=torch.int64, device=dev)
                out["primes"] = nprimes
        except torch.cuda.OutOfMemoryError:
            o = m = None
            torch.cuda.empty_cache()
            out["rows"].append({"t": t, "implicant_states": nm, "skipped": "%.1f GB of slice states (and the list) do not fit; %.1f GB "
                                "free, %.1f GB held by torch" % (need / 1e9, torch.cuda.mem_get_info()[0] / 1e9,
                                                                 torch.cuda.memory_reserved() / 1e9)})
            continue
        dqmc.dqmc_primes_sliced_multi(ctx.ctx, n, t, ttd, 0, o, m, lst, nprimes, count)  # warm-up
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            dqmc.dqmc_primes_sliced_multi(ctx.ctx, n, t, ttd, 0, o, m, lst, nprimes, count)
        end.record()
        torch.cuda.synchronize()
        assert int(count.item()) == nprimes
        ms = start.elapsed_time(end) / reps
        out["rows"].append({"t": t, "implicant_states": nm, "slices": 3**t, "slice_states_GB": need / 1e9,
                            "ms": ms, "cubes_per_s": 3**n / (ms / 1e3)})
        print("bench: sliced n=%d t=%d with %d implicant states %.1f ms" % (n, t, nm, ms), file=sys.stderr,
              flush=True)
        del o, m
        torch.cuda.empty_cache()
    del lst, ttd
    torch.cuda.empty_cache()
    return out


def bench_configs(ctx, n24_tt=None, n24_list=None, oracle_threads=0):
    """The smaller named workloads: n = 12 latency (median of 1000 calls) and
    n = 20 (median of 5), plus the host transfers the main step leaves out
    (truth table in, prime list out, pinned host memory).  With
    oracle_threads > 0 the oracle's O2 is timed on each whole workload as
    well, and its prime list is compared with the GPU's."""
    import numpy as np
    import torch

    from paper_2302_10083_amd import dqmc, inputs

    dev = ctx.torch_device
    out = {}
    for name, reps in (("c1_n12_bern05", 1000), ("c2a_n20_bern09", 5), ("c2b_n20_dnf200", 5)):
        spec = inputs.CONFIGS[name]
        n = spec["n"]
        tt = inputs.make(spec)
        ttd = ctx.tt_to_device(tt)
        state = ctx.new_state(n)
        count = torch.zeros(1, dtype=torch.int64, device=dev)
        dqmc.dqmc_primes(ctx.ctx, n, ttd, state, None, 0, count)
        torch.cuda.synchronize()
        c = int(count.item())
        lst = torch.empty(max(c, 1), dtype=torch.int64, device=dev)
        dqmc.dqmc_primes(ctx.ctx, n, ttd, state, lst, c, count)  # warm-up
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            dqmc.dqmc_primes(ctx.ctx, n, ttd, state, lst, c, count)
            b.record()
        torch.cuda.synchronize()
        ms = np.array([a.elapsed_time(b) for a, b in ev])
        med = float(np.median(ms))
        row = {"n": n, "primes": c, "reps": reps, "median_ms": med, "p90_ms": float(np.percentile(ms, 90)),
               "cubes_per_s": 3**n / (med / 1e3)}
        if n == 12:
            row["median_us"] = med * 1e3
        if oracle_threads > 0:
            det, ref = oracle_o2_seconds(n, tt, oracle_threads)
            row["oracle_O2"] = dict(det, threads=oracle_threads, cubes_per_s=3**n / det["total_s"],
                                    gpu_over_oracle=det["total_s"] / (med / 1e3),
                                    list_equal=bool(len(ref) == c and np.array_equal(
                                        lst[:c].cpu().numpy().view(np.uint64), ref)))
        out[name] = row
        print("bench: %s median %.4f ms" % (name, med), file=sys.stderr, flush=True)
        del state, lst
    if n24_tt is not None:
        # PCIe legs of the n = 24 workload, outside the timed step
        h_tt = torch.from_numpy(np.asarray(n24_tt, dtype=np.uint32).view(np.int32)).pin_memory()
        d_tt = torch.empty_like(h_tt, device=dev)
        h_list = torch.empty(n24_list.numel(), dtype=torch.int64, pin_memory=True)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        d_tt.copy_(h_tt, non_blocking=True)
        h_list.copy_(n24_list, non_blocking=True)
        torch.cuda.synchronize()
        a.record()
        d_tt.copy_(h_tt, non_blocking=True)
        b.record()
        torch.cuda.synchronize()
        ms_in = a.elapsed_time(b)
        a.record()
        h_list.copy_(n24_list, non_blocking=True)
        b.record()
        torch.cuda.synchronize()
        ms_out = a.elapsed_time(b)
        out["n24_host_transfers"] = {"tt_h2d_ms": ms_in, "tt_bytes": h_tt.numel() * 4, "list_d2h_ms": ms_out,
                                     "list_bytes": h_list.numel() * 8,
                                     "list_d2h_GBps": h_list.numel() * 8 / (ms_out / 1e3) / 1e9}
        print("bench: n=24 truth table in %.3f ms, list out %.2f ms" % (ms_in, ms_out), file=sys.stderr, flush=True)
        del d_tt, h_tt, h_list
    torch.cuda.empty_cache()
    return out


def bench_serving(nreq=2000, seed=25):
    """Serving mix (n in {10,14,18,22,25} with weights .4/.3/.15/.1/.05):
    saturation throughput from a closed loop, then Poisson arrivals at 0.5 and
    0.8 of it; latency = completion - submission on the server's clock.  The
    baseline serves the same arrival schedule one request at a time with one
    dqmc_primes launch sequence per request."""
    import threading

    import numpy as np
    import torch

    from paper_2302_10083_amd import dqmc, inputs

    specs = inputs.serving_specs(nreq, seed=seed)
    tts = [inputs.make(s) for s in specs]

    def run(srv, gaps):
        """Submit requests 0..len(gaps)-1 with the given gaps; a consumer
        thread waits for each in order and releases it."""
        k = len(gaps)
        ids, res = [], [None] * k

        def consumer():
            for i in range(k):
                while len(ids) <= i:
                    time.sleep(1e-4)
                res[i] = srv.wait(ids[i])
                srv.release(ids[i])

        th = threading.Thread(target=consumer)
        th.start()
        t0 = time.perf_counter()
        for s, tt, g in zip(specs[:k], tts[:k], gaps):
            if g > 0:
                time.sleep(g)
            ids.append(srv.submit(s["n"], tt))
        th.join()
        wall = time.perf_counter() - t0
        lat = np.array([r["t_done"] - r["t_submit"] for r in res])
        return wall, lat

    out = {"workload": "%d requests, n in {10,14,18,22,25} w.p. .4/.3/.15/.1/.05, half Bernoulli(0.5..0.95) "
                       "half DNF (seed %d)" % (nreq, seed)}
    print("bench: serving, %d requests generated" % nreq, file=sys.stderr, flush=True)
    with dqmc.Server(0) as srv:
        run(srv, [0.0] * 8)  # warm the pools and kernels
        wall, lat = run(srv, [0.0] * nreq)
        mu = nreq / wall
        out["saturation_jobs_per_s"] = mu
        print("bench: serving saturation %.1f jobs/s" % mu, file=sys.stderr, flush=True)
        rng = np.random.default_rng(seed)
        for frac in (0.5, 0.8):
            lam = frac * mu
            gaps = rng.exponential(1.0 / lam, size=nreq)
            wall, lat = run(srv, gaps)
            out["lambda_%.1f" % frac] = {"arrival_jobs_per_s": lam, "jobs_per_s": nreq / wall,
                                         "p50_ms": float(np.percentile(lat, 50) * 1e3),
                                         "p99_ms": float(np.percentile(lat, 99) * 1e3),
                                         "mean_ms": float(lat.mean() * 1e3)}
            print("bench: serving at %.1f of saturation done" % frac, file=sys.stderr, flush=True)
    # baseline: one request at a time, same arrivals at 0.5 mu
    ctx = dqmc.Context(0)
    dev = ctx.torch_device
    lam = 0.5 * mu
    arr = np.cumsum(np.random.default_rng(seed).exponential(1.0 / lam, size=nreq))
    lat = []
    t0 = time.perf_counter()
    for s, tt, a in zip(specs, tts, arr):
        now = time.perf_counter() - t0
        if now < a:
            time.sleep(a - now)
        n = s["n"]
        cap = min(3**n, max(1 << 18, 3 ** max(n - 3, 0) // 16))
        ttd = ctx.tt_to_device(tt)
        st = ctx.new_state(n)
        cnt = torch.zeros(1, dtype=torch.int64, device=dev)
        lst = torch.empty(cap, dtype=torch.int64, device=dev)
        dqmc.dqmc_primes(ctx.ctx, n, ttd, st, lst, cap, cnt)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - a)
        del st, lst
    ctx.close()
    torch.cuda.empty_cache()
    lat = np.array(lat)
    out["one_at_a_time_lambda_0.5"] = {"p50_ms": float(np.percentile(lat, 50) * 1e3),
                                       "p99_ms": float(np.percentile(lat, 99) * 1e3),
                                       "jobs_per_s": nreq / (time.perf_counter() - t0)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3_n24_dnf2000_noise")
    ap.add_argument("--cpu-sub-n", type=int, default=21,
                    help="the CPU baseline runs the oracle on f restricted to its first CPU_SUB_N variables")
    ap.add_argument("--cpu-threads", type=int, default=0, help="0: every core of the CPU share, at most 16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--tune-extra-groups", type=int, default=1,
                    help="pass plans with up to this many groups beyond the fewest are timed (autotuner)")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-cnf", action="store_true")
    ap.add_argument("--no-sparse", action="store_true")
    ap.add_argument("--no-sliced", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the prime-implicant path has no "
              "multi-GPU mode (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2302_10083_amd import dqmc, inputs

    spec = inputs.CONFIGS[args.workload]
    n = spec["n"]
    tt = inputs.make(spec)
    ctx = dqmc.Context(0)
    dev = ctx.torch_device
    ttd = ctx.tt_to_device(tt)
    state = ctx.new_state(n)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    print("bench: n=%d workload=%s state=%.2f GB" % (n, args.workload, state.numel() * 4 / 1e9),
          file=sys.stderr, flush=True)
    # size the list with a count-only run
    dqmc.dqmc_primes(ctx.ctx, n, ttd, state, None, 0, count)
    torch.cuda.synchronize()
    nprimes = int(count.item())
    lst = torch.empty(max(nprimes, 1), dtype=torch.int64, device=dev)
    print("bench: %d primes (list %.2f GB)" % (nprimes, nprimes * 8 / 1e9), file=sys.stderr, flush=True)
    # the autotuner times the pass plans on this input and keeps the fastest
    plan_trials = []
    if not args.no_tune and n > 12:
        plan_trials = dqmc.dqmc_plan_autotune(ctx.ctx, n, ttd, state, count, extra_groups=args.tune_extra_groups,
                                              reps=1)
        print("bench: plan autotune: %d trials, chosen %s%s" % (len(plan_trials), dqmc.dqmc_get_plan(ctx.ctx, n),
                                                                 " with the top-digit split"
                                                                 if dqmc.dqmc_get_split(ctx.ctx, n) else ""),
              file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        dqmc.dqmc_primes(ctx.ctx, n, ttd, state, lst, nprimes, count)
    torch.cuda.synchronize()

    dqmc.dqmc_profile(ctx.ctx, True)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        dqmc.dqmc_primes(ctx.ctx, n, ttd, state, lst, nprimes, count)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    recs = dqmc.dqmc_profile_read(ctx.ctx)
    dqmc.dqmc_profile(ctx.ctx, False)
    assert int(count.item()) == nprimes
    ms_step = start.elapsed_time(end) / args.steps
    cubes = 3**n

    # per-pass figures (average over the timed steps)
    passes = {}
    for r in recs:
        p = passes.setdefault(r["pass_name"], dict(ms=0.0, k=0, model_bytes=r["model_bytes"],
                                                   lbpp=r["list_bytes_per_prime"]))
        p["ms"] += r["ms"]
        p["k"] += 1
    # With the row and chunk flags (n = 24, plan [6, 6]) the reduce of digits
    # 13..18 and the final reduce move data-dependent bytes: the rows and runs
    # the flags select, counted from the flags of the last step.  Their dense
    # model (every word read and written) is kept as dense_model_GB.
    units = dqmc.dqmc_flag_units(ctx.ctx) if n == 24 else {"used": False}
    ntiles = 3 ** max(n - 12, 0)
    flagged = {}
    if units["used"]:
        flag_bytes = 4.0 * 729 * 274 * 23
        flagged["col_reduce_g13_6"] = 2.0 * units["reduce13_rows_bytes"] + flag_bytes
        flagged["low_reduce_count"] = (units["final_runs_bytes"] + units["final_store_bytes"]
                                       + ntiles * 4.0 * (2 * 9 + 1))  # flags, chunk map, count
    pass_rows = []
    total_bytes = 0.0
    for name, p in passes.items():
        ms = p["ms"] / p["k"]
        dense = p["model_bytes"] + p["lbpp"] * nprimes
        b = flagged.get(name, dense)
        total_bytes += b
        row = dict(name=name, ms=round(ms, 4), model_GB=round(b / 1e9, 3), GBps=round(b / (ms / 1e3) / 1e9, 1))
        if name in flagged:
            row["dense_model_GB"] = round(dense / 1e9, 3)
        pass_rows.append(row)
    dom = max(pass_rows, key=lambda r: r["ms"])
    dom_bytes = dom["model_GB"] * 1e9
    achieved = dom_bytes / (dom["ms"] / 1e3) / 1e9
    traffic = read_traffic(dom["name"], args.workload)

    out = {
        "metric": "ternary cubes/s (DenseQMC primes at n=%d: truth table -> prime bitmap + sorted list)" % n,
        "value": cubes / (ms_step / 1e3),
        "unit": "cubes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "cubes": cubes, "truth_table": spec,
                   "primes": nprimes, "layout": "H5 (243 cubes per 256-bit block)", "parallelism": "single-gpu"},
        "hbm_GBps_model": total_bytes / (ms_step / 1e3) / 1e9,
        "hbm_frac_model": total_bytes / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBPS,
        "model_bytes_per_step": total_bytes,
        "flag_units": units,
        "wall_s_timed": wall,
        "passes": pass_rows,
        "plan": {"groups": dqmc.dqmc_get_plan(ctx.ctx, n), "passes_per_step": len(pass_rows),
                 "split_top_digit": dqmc.dqmc_get_split(ctx.ctx, n),
                 "autotune_trials": [["split" if t["split"] else t["sizes"], round(t["ms"], 3)]
                                     for t in plan_trials]},
        # achieved: the pass's model bytes per second (for the flagged passes
        # the bytes their flags select, else every word the plan reads and
        # writes); traffic: HBM bytes by rocprofv3 counters for these sources
        "roofline": {"bound": "hbm", "kernel": dom["name"], "achieved": achieved, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic, "model_bytes_per_launch": dom_bytes,
                     "traffic_GBps": traffic / (dom["ms"] / 1e3) / 1e9 if traffic else None,
                     "frac_traffic": traffic / (dom["ms"] / 1e3) / 1e9 / HBM_PEAK_GBPS if traffic else None},
        "paper_context": {"n24_seconds_one_core": PAPER_N24_SECONDS,
                          "n24_cubes_per_s": cubes / PAPER_N24_SECONDS if n == 24 else None},
    }

    if not args.no_cpu_baseline:
        threads = baseline_threads(args.cpu_threads)
        print("bench: oracle O2 on the %d-variable restriction, %d threads" % (min(args.cpu_sub_n, n), threads),
              file=sys.stderr, flush=True)
        rate, used, det, sub_tt, sub_primes = cpu_baseline(n, tt, args.cpu_sub_n, threads)
        sub_n = min(args.cpu_sub_n, n)
        # the restriction's primes double as a parity check of the GPU path
        sub_ttd = ctx.tt_to_device(sub_tt)
        sub_state = ctx.new_state(sub_n)
        sub_count = torch.zeros(1, dtype=torch.int64, device=dev)
        sub_list = torch.empty(max(len(sub_primes), 1), dtype=torch.int64, device=dev)
        dqmc.dqmc_primes(ctx.ctx, sub_n, sub_ttd, sub_state, sub_list, len(sub_primes), sub_count)
        torch.cuda.synchronize()
        same = (int(sub_count.item()) == len(sub_primes) and
                np.array_equal(sub_list[:len(sub_primes)].cpu().numpy().view(np.uint64), sub_primes))
        del sub_ttd, sub_state, sub_list
        out["cpu_baseline"] = {"value": rate, "unit": "cubes/s", "cores": used, "kind": "oracle",
                               "variant": "O2 (M sweep by the Lemma of Sec. 4.1, then the O formula)",
                               "sample": "O2 of the n=%d workload restricted to x%d..x%d = 0: a %d-variable "
                                         "function, the first 3^%d cubes of its cube space; %.1f s" %
                                         (n, sub_n + 1, n, sub_n, sub_n, det["total_s"]),
                               "seconds": det, "host": host_info(),
                               "gpu_over_cpu": (cubes / (ms_step / 1e3)) / rate}
        out["sample_parity"] = {"function": "restriction to x%d..x%d = 0" % (sub_n + 1, n), "n": sub_n,
                                "oracle_primes": det["primes"], "gpu_equal": bool(same)}
    if not args.no_cnf:
        # CNF of a sparse function: the primes of its complement, with the
        # complement taken as the table is loaded (DQMC_NEGATE).  The sparse
        # function here is NOT f, so its CNF clauses are f's primes.
        sparse = ~np.asarray(tt, dtype=np.uint32)
        sd = ctx.tt_to_device(sparse)
        for _ in range(args.warmup):
            dqmc.dqmc_primes_ex(ctx.ctx, n, sd, dqmc.DQMC_NEGATE, state, lst, nprimes, count)
        torch.cuda.synchronize()
        start.record()
        for _ in range(args.steps):
            dqmc.dqmc_primes_ex(ctx.ctx, n, sd, dqmc.DQMC_NEGATE, state, lst, nprimes, count)
        end.record()
        torch.cuda.synchronize()
        ms_cnf = start.elapsed_time(end) / args.steps
        out["cnf"] = {"workload": "CNF of NOT(%s) (density %.4f): primes of its complement" %
                                  (args.workload, float(np.unpackbits(sparse.view(np.uint8)).mean())),
                      "ms": ms_cnf, "cubes_per_s": cubes / (ms_cnf / 1e3), "clauses": int(count.item()),
                      "clauses_equal_dnf_primes": int(count.item()) == nprimes}
        del sd
        print("bench: cnf %.2f ms" % ms_cnf, file=sys.stderr, flush=True)
    if not args.no_configs:
        out["configs"] = bench_configs(ctx, tt if n == 24 else None, lst[:nprimes] if n == 24 else None,
                                       0 if args.no_cpu_baseline else baseline_threads(args.cpu_threads))
    if not args.no_batch or not args.no_sparse or not args.no_sliced:
        del lst, state
        torch.cuda.empty_cache()
    if not args.no_sliced:
        out["sliced"] = bench_sliced(ctx)
        out["sliced_n27"] = bench_sliced(ctx, "c3x_n27_dnf2000_noise", ts=((3, 1), (3, 4)), reps=1)
    if not args.no_sparse:
        out["sparse"] = bench_sparse(ctx)
        print("bench: sparse %s" % ", ".join("d=%.2f %.1f ms (dense %.1f ms)" % (r["density"], r["ms_sparse"],
                                                                              r["ms_dense"])
                                              for r in out["sparse"]["rows"]), file=sys.stderr, flush=True)
    if not args.no_batch:
        out["batch"] = bench_batch(ctx)
        print("bench: batch %.2f ms (%.0f fns/s), per-function launches %.2f ms" % (
            out["batch"]["ms"], out["batch"]["fns_per_s"], out["batch"]["per_fn_launch_ms"]), file=sys.stderr, flush=True)

    if not args.no_serving:
        torch.cuda.empty_cache()
        out["serving"] = bench_serving(args.serving_requests)
        sv = out["serving"]
        print("bench: serving saturation %.1f jobs/s; p99 %.1f ms at 0.8 of it" % (
            sv["saturation_jobs_per_s"], sv["lambda_0.8"]["p99_ms"]), file=sys.stderr, flush=True)

    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
