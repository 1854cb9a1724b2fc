"""Benchmark: factorizations per second of the bounded lexicographic
enumeration on one MI355X.

One step = the whole path over the d=6 query (generators drawn from seed 0,
n = 100000, |Z| = 31,970,991,953): a count-mode enumeration of all of Z, then a
store-mode enumeration of its 5e8 lex-smallest elements into a device buffer
(12 GB).  Each call runs the count table, the slice bounds, the walker and the
finalize kernels.  value = (|Z| + 5e8) / step time.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-batch] [--no-served]

Beside the step, the same run measures (timed on their own, not part of the
step): the 4096-query mixed batch in one launch ("batch"), and the served
stream of 20000 queries through the request server against one launch per
query ("served": closed-loop queries/s, p50/p99 latency at open-loop Poisson
arrivals of half and nine tenths of that rate).

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks.  The walker's count mode is integer-ALU work.  The
# published fp32 vector rate, 157.3 TFLOP/s = 2 FLOP x 128 lanes per CU per
# cycle x 256 CUs x 2.4 GHz, gives the vector lane rate: 128 x 256 x 2.4e9 =
# 7.86e13 int32 lane-ops/s (fz_probe_int_valu measures ~7.5e13 for 32-bit
# adds on the device).
PEAK_INT32_OPS = 128 * 256 * 2.4e9
PEAK_HBM_BYTES = 8.0e12
# Algorithmic int32 work of the count walker (stated with the derivation in
# the design notes): per element, advance the last pair, test a_d >= 0 and
# count = 3 ops; per lane prefix, split the remainder (4), look up the residue
# class (1), solve the pair (1), range-test (1) and the failing test that
# ends the progression (1) = 8 ops.
OPS_PER_ELEMENT = 3
OPS_PER_PREFIX = 8


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_enum_d6_n100000.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2405_07989_amd", "csrc", "fz_kernels.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of each walker from the committed rocprofv3 PMC
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size);
    None when the file is missing or the walker source changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            line = line.strip()
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return {k: float(v) for k, v in vals.items() if k.endswith("_bytes")}


def host_threads():
    """Host cores this process may use: its CPU affinity, capped by
    OMP_NUM_THREADS when that is set (a GPU machine's share of its host)."""
    n = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(omp))) if omp.isdigit() and int(omp) > 0 else n


def cpu_baseline(n, g, N, cpu_seconds=20.0, windows=256):
    """The oracle's plain ascending walk, timed on windows spread over the
    whole set: window j starts at the element of rank about j N / windows
    (from the oracle's own unranking) and walks k elements from there, 3/4 of
    the windows with the count consumer and 1/4 with the store consumer.  The
    windows run on every host core this process has (one walk per thread;
    the C oracle releases the interpreter lock), sized to about cpu_seconds
    of single-core work; the single-core rate on the first windows is
    reported beside it."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    starts = [oracle.unrank_dp(n, g, (j * N) // windows + (N // windows) // 2)
              for j in range(windows)]
    # single-core rate on a few windows of 1e6 elements
    t0 = time.perf_counter()
    probe = 0
    for j in range(0, windows, windows // 4):
        probe += oracle.walk(n, g, start=starts[j], stop_after=10**6)["count"]
    single_rate = probe / (time.perf_counter() - t0)
    k = max(10**5, int(single_rate * cpu_seconds / windows))

    def one(j):
        if j % 4 == 3:
            return len(oracle.walk(n, g, start=starts[j], stop_after=k, out_cap=k)["store"])
        return oracle.walk(n, g, start=starts[j], stop_after=k)["count"]

    threads = host_threads()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        got = list(ex.map(one, range(windows)))
    dt = time.perf_counter() - t0
    total = sum(got)
    assert all(x == k for x in got[:-1])  # every window but the last holds k elements
    return dict(value=total / dt, unit="factorizations/s", cores=threads, kind="oracle",
                single_core_value=single_rate,
                sample=(f"{windows} windows of {k} elements each, starting at ranks "
                        f"(j + 1/2) |Z| / {windows} of the same d=6 query (3/4 count consumer, "
                        f"1/4 store consumer), {total} elements in {dt:.1f} s on {threads} "
                        f"threads; C oracle, plain ascending nested loops"))


def percentile(v, p):
    v = sorted(v)
    if not v:
        return None
    k = max(0, min(len(v) - 1, int(math.ceil(p * len(v))) - 1))
    return v[k]


def measure_batch(fz, reps=3, autotune=True):
    """The 4096-query mixed batch (count / histogram / predicate) as one
    fz_batch call; median of reps, every result checked against the stored
    counts."""
    import fzinputs
    w = fzinputs.load_golden()["batch"]["queries"]
    qs = [dict(n=q["n"], g=q["g"], mode=q["mode"], target_len=q["target_len"]) for q in w]
    fz.batch(qs[:64])

    def timed(label):
        times, walk, prep = [], [], []
        for r in range(reps):
            fz.profile_reset()
            fz.profile_enable(True)
            t0 = time.perf_counter()
            res = fz.batch(qs)
            times.append(time.perf_counter() - t0)
            fz.profile_enable(False)
            st = fz.last_stats()
            prep.append(fz.profile_read("batch.tables")[0] + fz.profile_read("batch.slices")[0])
            walk.append(fz.profile_read("batch.walk")[0])
            for q, x, ww in zip(qs, res, w):
                ok = x["status"] == 0 and (x["count"] == ww["count"] or
                                           (q["mode"] == "exists" and x["found"]))
                if not ok:
                    raise RuntimeError(f"batch: wrong result for {q}: {x}")
            log(f"batch ({label}) rep {r + 1}/{reps}: {times[-1] * 1e3:.1f} ms")
        t = sorted(times)[len(times) // 2]
        wk = sorted(walk)[len(walk) // 2]
        # the walker's algorithmic int32 work, as for the single query
        ops = OPS_PER_ELEMENT * st["elements"] + OPS_PER_PREFIX * st["prefixes"]
        return {"ms": t * 1e3, "queries_per_s": len(qs) / t,
                "factorizations_per_s": elements / t,
                "prep_ms": sorted(prep)[len(prep) // 2], "walk_ms": wk,
                "walker_stats": st,
                "roofline": {"bound": "alu", "achieved": ops / (wk / 1e3) / 1e12,
                             "peak": PEAK_INT32_OPS / 1e12, "unit": "Tops/s (int32)",
                             "frac": ops / (wk / 1e3) / PEAK_INT32_OPS, "ops": ops}}

    elements = sum(x["count"] for x in w)
    out = {"queries": len(qs),
           "workload": "4096 queries: d in 3..8, generators in [5,1000], n log-uniform in "
                       "[1e3,1e6], |Z| <= 1e8, consumer count/hist/exists"}
    out["default"] = timed("default slices")
    if not autotune:
        out.update({k: out["default"][k] for k in ("ms", "queries_per_s", "factorizations_per_s",
                                                    "prep_ms", "walk_ms")})
        return out
    # the autotuner picks slices per wave and workgroups per CU on this batch
    tune = fz.autotune(qs, reps=1)
    out["autotune"] = {k: tune[k] for k in ("slices_per_wave", "workgroups_per_cu", "candidates")}
    try:
        out["tuned"] = timed("tuned")
    finally:
        fz.config_set("slices_per_wave", 0)
        fz.config_set("workgroups_per_cu", 0)
    best = min(out["default"], out["tuned"], key=lambda x: x["ms"])
    out.update({k: best[k] for k in ("ms", "queries_per_s", "factorizations_per_s", "prep_ms",
                                     "walk_ms")})
    return out


def measure_single_small(fz, torch, reps=200):
    """End-to-end latency of the small single query (g = (11,13,17,23),
    n = 10000, |Z| = 3,009,519), host call to host return: the count, and
    the store of all its rows into a preallocated device tensor (48 MB)."""
    import fzinputs
    w = fzinputs.load_golden()["single_small"]
    n, g, N = w["n"], w["g"], w["count"]
    out = torch.empty((N, len(g)), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    res = {"workload": f"g={g} n={n}: count |Z|={N}; store all {N} rows ({N * len(g) * 4} B)"}
    for mode in ("count", "store"):
        lat = []
        for r in range(reps + 10):
            t0 = time.perf_counter()
            if mode == "count":
                ok = fz.count(n, g) == N
            else:
                ok = fz.enumerate_device(n, g, out) == (N, N)
            dt = time.perf_counter() - t0
            if not ok:
                raise RuntimeError(f"single small query: wrong {mode} result")
            if r >= 10:
                lat.append(dt)
        res[f"{mode}_p50_us"] = percentile(lat, 0.5) * 1e6
        res[f"{mode}_p99_us"] = percentile(lat, 0.99) * 1e6
        res[f"{mode}_factorizations_per_s"] = N / percentile(lat, 0.5)
    del out
    return res


def measure_variant(fz, n, g, N, ls, reps=3):
    """The variant walk (knob "variant" = 1; not the metric): the count of the
    d=6 query in drawn and in descending generator order and the length-set
    histogram, with the common-divisor skip over the last two and three
    generators and closed-form run lengths.  Kernel time of the walker,
    results checked against the stored counts."""
    out = {"what": "common-divisor skip over the last 2 and 3 generators (Sec. 3.2.4) + "
                   "closed-form run lengths; reported beside the metric, not as it"}
    fz.config_set("variant", 1)
    try:
        for label, order, fn, key, want in [
                ("count_drawn_order", 1, lambda: fz.count(n, g), "enum.count", N),
                ("count_descending_order", 0, lambda: fz.count(n, g), "enum.count", N),
                ("length_set_hist", 0, lambda: int(fz.length_hist(ls["n"], ls["g"])[0].sum()),
                 "enum.hist", ls["count"])]:
            fz.config_set("walk_order", order)
            fn()
            fz.profile_reset()
            fz.profile_enable(True)
            for _ in range(reps):
                if fn() != want:
                    raise RuntimeError(f"variant walk: wrong result ({label})")
            fz.profile_enable(False)
            ms, k = fz.profile_read(key)
            st = fz.last_stats()
            out[label] = {"avg_launch_ms": ms / max(k, 1),
                          "factorizations_per_s": want / (ms / 1e3 / max(k, 1)),
                          "rows": st["rows"], "prefixes": st["prefixes"]}
    finally:
        fz.config_set("variant", 0)
        fz.config_set("walk_order", 0)
    return out


def _serve(fz, qs, gaps=None, inflight=4):
    """Submits qs through one server (at the arrival gaps, or all at once),
    collects every result on a second thread, and returns (elapsed s, server
    stats, results)."""
    import threading
    import queue as qmod
    srv = fz.Server(max_inflight=inflight)
    pending = qmod.Queue()
    results = [None] * len(qs)

    def collector():
        while True:
            item = pending.get()
            if item is None:
                return
            i, t = item
            results[i] = srv.wait(t)

    th = threading.Thread(target=collector)
    th.start()
    t0 = time.perf_counter()
    next_t = t0
    for i, q in enumerate(qs):
        if gaps is not None:
            next_t += gaps[i]
            dt = next_t - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
        # outputs were allocated (torch.empty, no kernel) and synchronized up front
        pending.put((i, srv.submit(q, sync=False)))
    pending.put(None)
    th.join()
    elapsed = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    return elapsed, st, results


def measure_served(fz, torch, n_single=1000):
    """The served stream: saturation (all 20000 queries offered at once),
    then open-loop Poisson arrivals at 0.5x and 0.9x of the saturation rate;
    one launch per query (the single-query entry points, sequentially) on the
    first n_single queries of the same stream."""
    import fzinputs
    golden = fzinputs.load_golden()
    counts = golden["served"]["counts"]
    stream = fzinputs.served_stream(golden)
    # every store query's output buffer (|Z| rows) is allocated up front
    for i, q in enumerate(stream):
        if q["mode"] == "store":
            q["out"] = torch.empty((max(counts[i], 1), len(q["g"])), dtype=torch.int32,
                                   device="cuda")
            q["max_tuples"] = counts[i]
    torch.cuda.synchronize()

    def result_ok(q, r, c):
        if q["mode"] == "store":
            return r["status"] == 0 and r["total"] == c == r["written"]
        return r["status"] == 0 and (r["count"] == c or (q["mode"] == "exists" and r["found"]))

    def check(results, label):
        for i, (q, r) in enumerate(zip(stream, results)):
            if not result_ok(q, r, counts[i]):
                raise RuntimeError(f"served ({label}): wrong result for query {i} {q}: {r}")

    _serve(fz, stream[:500])  # warm-up: buffers of the slots
    elapsed, st, res = _serve(fz, stream)
    check(res, "saturation")
    qps = len(stream) / elapsed
    log(f"served saturation: {qps:.0f} queries/s, p50 {st['p50_us']:.0f} us, "
        f"p99 {st['p99_us']:.0f} us")
    out = {"queries": len(stream), "store_queries": golden["served"]["n_store"],
           "saturation": {"queries_per_s": qps, "p50_us": st["p50_us"], "p99_us": st["p99_us"],
                          "mean_batch": st["mean_batch"], "launches": st["launches"]}}
    for frac in (0.5, 0.9):
        gaps = fzinputs.exponential_gaps(11, frac * qps, len(stream))
        el, st, res = _serve(fz, stream, gaps=gaps)
        check(res, f"open loop {frac}")
        out[f"open_loop_{frac}"] = {"offered_qps": frac * qps, "achieved_qps": len(stream) / el,
                                    "p50_us": st["p50_us"], "p99_us": st["p99_us"],
                                    "max_us": st["max_us"], "mean_batch": st["mean_batch"]}
        log(f"served open loop at {frac} x: p50 {st['p50_us']:.0f} us, p99 {st['p99_us']:.0f} us")
    # one launch per query
    lat = []
    t0 = time.perf_counter()
    for i, q in enumerate(stream[:n_single]):
        t1 = time.perf_counter()
        if q["mode"] == "count":
            c = fz.count(q["n"], q["g"])
        elif q["mode"] == "hist":
            c = int(fz.length_hist(q["n"], q["g"])[0].sum())
        elif q["mode"] == "exists":
            fz.exists(q["n"], q["g"], q["target_len"])
            c = counts[i]  # the predicate reports no count
        else:
            c, _ = fz.enumerate_device(q["n"], q["g"], q["out"])
        lat.append(time.perf_counter() - t1)
        if c != counts[i]:
            raise RuntimeError(f"one launch per query: wrong count for query {i}")
    single_qps = n_single / (time.perf_counter() - t0)
    log(f"one launch per query: {single_qps:.0f} queries/s")
    out["one_launch_per_query"] = {"queries": n_single, "queries_per_s": single_qps,
                                   "p50_us": percentile(lat, 0.5) * 1e6,
                                   "p99_us": percentile(lat, 0.99) * 1e6}
    out["speedup_vs_one_launch_per_query"] = qps / single_qps
    # one fz_batch call per query (a batch of one), the same queries
    lat_b = []
    t0 = time.perf_counter()
    for i, q in enumerate(stream[:n_single]):
        t1 = time.perf_counter()
        r = fz.batch([q])[0]
        lat_b.append(time.perf_counter() - t1)
        if not result_ok(q, r, counts[i]):
            raise RuntimeError(f"batch of one: wrong result for query {i} {q}: {r}")
    batch1_qps = n_single / (time.perf_counter() - t0)
    log(f"one fz_batch call per query: {batch1_qps:.0f} queries/s")
    out["one_batch_call_per_query"] = {"queries": n_single, "queries_per_s": batch1_qps,
                                       "p50_us": percentile(lat_b, 0.5) * 1e6,
                                       "p99_us": percentile(lat_b, 0.99) * 1e6}
    out["speedup_vs_one_batch_call_per_query"] = qps / batch1_qps
    out["workload"] = ("20000 queries drawn as the batch, 20% store queries (|Z| <= 1e7, "
                       "written to device buffers allocated before timing), up to 4 launches "
                       "in flight")
    for q in stream:
        q.pop("out", None)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the batch with the default slices only (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed steps, copy 1 GiB device to device 3 times (the "
                         "reference kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import fzinputs
    import paper_2405_07989_amd as fz

    w = fzinputs.load_golden()["single_large"]
    n, g, M, N = w["n"], w["g"], w["store_max_tuples"], w["count"]
    assert g == fzinputs.single_large_generators(w["seed"])
    torch.cuda.set_device(0)
    out = torch.empty((M, len(g)), dtype=torch.int32, device="cuda")
    log(f"workload: n={n} g={g} |Z|={N} store rows={M}")

    # The workload keeps the generators in drawn order: the count walks in
    # that order too (the library would otherwise walk order-free consumers
    # in descending generator order, timed separately below).
    fz.config_set("walk_order", 1)

    def step():
        c = fz.count(n, g)
        st_count = fz.last_stats()
        total, written = fz.enumerate_device(n, g, out)
        if c != N or total != N or written != M:
            raise RuntimeError(f"wrong result: count {c}, total {total}, written {written}")
        return st_count

    for i in range(args.warmup):
        step()
        log(f"warmup {i + 1}/{args.warmup} done")

    fz.profile_reset()
    fz.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        st = step()
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    fz.profile_enable(False)

    ms_step = elapsed * 1e3 / args.steps
    value = (N + M) / (elapsed / args.steps)
    valu_probe = fz.probe_int_valu()  # after the timed steps
    log(f"int32 add probe: {valu_probe['lane_ops_per_s'] / 1e12:.2f} Tops/s")
    write_probe = fz.probe_hbm_write(M * 4 * len(g))  # as many bytes as the store writes
    log(f"HBM write probe: {write_probe['bytes_per_s'] / 1e9:.0f} GB/s")
    kt = {k: fz.profile_read(k) for k in ["dp", "restab", "slices", "enum.count", "enum.store",
                                          "finalize"]}
    cnt_ms, cnt_n = kt["enum.count"]
    sto_ms, sto_n = kt["enum.store"]
    avg_count_s = cnt_ms / 1e3 / max(cnt_n, 1)
    avg_store_s = sto_ms / 1e3 / max(sto_n, 1)
    ops = OPS_PER_ELEMENT * st["elements"] + OPS_PER_PREFIX * st["prefixes"]
    achieved = ops / avg_count_s
    store_bytes = M * len(g) * 4
    store_bw = store_bytes / avg_store_s

    res = {
        "metric": "factorizations/s (count+store mode)",
        "value": value,
        "unit": "factorizations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded generators, no dataset)",
        "config": {
            "workload": (f"d=6 generators {g} (SplitMix64 seed {w['seed']}), n={n}: count all "
                         f"|Z|={N} + store the {M} lex-smallest elements on the device"),
            "n": n, "g": g, "count": N, "store_rows": M,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "fz_enum_kernel<M=3,count>",
            "achieved": achieved / 1e12,
            "peak": PEAK_INT32_OPS / 1e12,
            "unit": "Tops/s (int32)",
            "frac": achieved / PEAK_INT32_OPS,
            "traffic": None,
            "ops_per_launch": ops,
            "avg_launch_ms": avg_count_s * 1e3,
            # the device's own sustained int32 add rate (fz_probe_int_valu)
            "measured_int_add_peak": valu_probe["lane_ops_per_s"] / 1e12,
        },
        "store_roofline": {
            "bound": "hbm",
            "kernel": "fz_enum_kernel<M=3,store>",
            "achieved": store_bw / 1e9,
            "peak": PEAK_HBM_BYTES / 1e9,
            "unit": "GB/s",
            "frac": store_bw / PEAK_HBM_BYTES,
            "traffic": None,
            "avg_launch_ms": avg_store_s * 1e3,
            # the device's own sustained write rate (fz_probe_hbm_write,
            # 16-byte stores, same byte count)
            "measured_write_peak": write_probe["bytes_per_s"] / 1e9,
        },
        "count_factorizations_per_s": N / avg_count_s,
        "store_factorizations_per_s": M / avg_store_s,
        "kernel_ms_per_step": {k: v[0] / max(args.steps, 1) for k, v in kt.items()},
        "walker_stats": st,
    }
    # the same count in the library's default (descending) walk order
    fz.config_set("walk_order", 0)
    fz.count(n, g)
    fz.profile_reset()
    fz.profile_enable(True)
    for _ in range(max(args.steps, 1)):
        if fz.count(n, g) != N:
            raise RuntimeError("wrong count in descending walk order")
    fz.profile_enable(False)
    st_desc = fz.last_stats()
    desc_ms, desc_n = fz.profile_read("enum.count")
    res["count_descending_walk_order"] = {
        "avg_launch_ms": desc_ms / max(desc_n, 1),
        "factorizations_per_s": N / (desc_ms / 1e3 / max(desc_n, 1)),
        "ops_per_launch": OPS_PER_ELEMENT * st_desc["elements"] +
                          OPS_PER_PREFIX * st_desc["prefixes"],
        "walker_stats": st_desc,
    }
    # The length-set workload (d = 11, a repeated generator): its length
    # histogram, timed on its own (not part of the step).
    import fzinputs
    ls = fzinputs.load_golden()["length_set"]
    fz.length_hist(ls["n"], ls["g"])
    fz.profile_reset()
    fz.profile_enable(True)
    for _ in range(max(args.steps, 1)):
        h, _, _ = fz.length_hist(ls["n"], ls["g"])
        if int(h.sum()) != ls["count"]:
            raise RuntimeError("wrong length-set histogram")
    fz.profile_enable(False)
    st_ls = fz.last_stats()
    ls_ms, ls_n = fz.profile_read("enum.hist")
    res["length_set_hist"] = {
        "workload": f"d={len(ls['g'])} g={ls['g']} n={ls['n']}: histogram of lengths "
                    f"({ls['nbins']} bins) of |Z|={ls['count']}",
        "avg_launch_ms": ls_ms / max(ls_n, 1),
        "factorizations_per_s": ls["count"] / (ls_ms / 1e3 / max(ls_n, 1)),
        "walker_stats": st_ls,
    }
    log("length-set histogram done")
    res["variant_walk"] = measure_variant(fz, n, g, N, ls)
    log("variant walk: count drawn %.2f ms, length-set histogram %.1f ms" % (
        res["variant_walk"]["count_drawn_order"]["avg_launch_ms"],
        res["variant_walk"]["length_set_hist"]["avg_launch_ms"]))
    res["single_small"] = measure_single_small(fz, torch)
    log("single small query: count p50 %.0f us, store p50 %.0f us" % (
        res["single_small"]["count_p50_us"], res["single_small"]["store_p50_us"]))
    del out
    torch.cuda.empty_cache()
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.int32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()
        log("copy calibration done (3 x 1 GiB)")
    if not args.no_batch:
        log("batch (4096 queries) ...")
        res["batch"] = measure_batch(fz, autotune=not args.no_autotune)
    if not args.no_served:
        log("served stream (20000 queries) ...")
        res["served"] = measure_served(fz, torch)
    tr = measured_traffic()
    if tr:
        res["roofline"]["traffic"] = tr.get("count_walker_bytes")
        res["store_roofline"]["traffic"] = tr.get("store_walker_bytes")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        res["cpu_baseline"] = cpu_baseline(n, g, N)
        log("cpu baseline done")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
