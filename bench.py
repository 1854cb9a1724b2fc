"""Benchmark: factorizations per second of the bounded lexicographic
enumeration on one MI355X.

One step = the whole path over the d=6 query (generators drawn from seed 0,
n = 100000, |Z| = 31,970,991,953): a count-mode enumeration of all of Z, then a
store-mode enumeration of its 5e8 lex-smallest elements into a device buffer
(12 GB).  Each call runs the count table, the slice bounds, the walker and the
finalize kernels.  value = (|Z| + 5e8) / step time.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks.  The walker's count mode is integer-ALU work: 256
# CUs x 4 SIMD x 16 lanes x 2.4 GHz = 3.93e13 int32 lane-ops/s.
PEAK_INT32_OPS = 256 * 4 * 16 * 2.4e9
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


def cpu_baseline(n, g, seconds_target=15.0):
    """The oracle's ascending walk on the lex-smallest elements of the same
    query (count consumer, then store consumer), one host core."""
    import oracle
    import numpy as np  # noqa: F401

    k = 2_000_000
    t0 = time.perf_counter()
    oracle.walk(n, g, stop_after=k)
    dt = time.perf_counter() - t0
    # scale the sample to about seconds_target of CPU time, split count/store
    k_count = max(k, int(k * (0.6 * seconds_target) / max(dt, 1e-3)))
    k_store = max(k, int(k * (0.4 * seconds_target) / max(dt, 1e-3)) // 2)
    t0 = time.perf_counter()
    c = oracle.walk(n, g, stop_after=k_count)["count"]
    t1 = time.perf_counter()
    s = oracle.walk(n, g, stop_after=k_store, out_cap=k_store)["store"]
    t2 = time.perf_counter()
    assert c == k_count and len(s) == k_store
    rate = (k_count + k_store) / (t2 - t0)
    return dict(value=rate, unit="factorizations/s", cores=1, kind="oracle",
                sample=(f"lex-smallest {k_count} elements (count consumer, {t1 - t0:.1f}s) + "
                        f"lex-smallest {k_store} elements (store consumer, {t2 - t1:.1f}s) "
                        f"of the same d=6 query, single-threaded C oracle"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
        },
        "count_factorizations_per_s": N / avg_count_s,
        "store_factorizations_per_s": M / avg_store_s,
        "kernel_ms_per_step": {k: v[0] / max(args.steps, 1) for k, v in kt.items()},
        "walker_stats": st,
    }
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
    tr = measured_traffic()
    if tr:
        res["roofline"]["traffic"] = tr.get("count_walker_bytes")
        res["store_roofline"]["traffic"] = tr.get("store_walker_bytes")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        res["cpu_baseline"] = cpu_baseline(n, g)
        log("cpu baseline done")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
