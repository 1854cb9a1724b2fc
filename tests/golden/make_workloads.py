"""Write tests/golden/workloads.json: the choices that need a count, and the
expected values the tests compare against.  Calls only the CPU oracle.

    python tests/golden/make_workloads.py

Choices (the readings of the workload descriptions):
  single_small   g = (11,13,17,23), n = 10000.
  single_large   d = 6 generators from SplitMix64(seed), distinct, uniform in
                 [20,200], gcd 1, drawn order, n = 100000; seed = the first of
                 0,1,2,... whose |Z| lies in [1e10, 1e11].  Store mode keeps the
                 5e8 lex-smallest elements.
  length_set     10 distinct generators uniform in [50,500] with gcd 1 from
                 SplitMix64(0), then a copy of one of them; n = the smallest n
                 with |Z(n)| >= 1e11.
  batch          4096 queries; query i draws from SplitMix64(i-th output of
                 SplitMix64(master)) and draws again while |Z| > 1e8.
  served         20000 queries drawn like the batch, 20% of them store
                 queries; a draw is redrawn while |Z| > 1e8, or > 1e7 for a
                 store query.  Kept: each query's seed-derived redraw count
                 (fzinputs.served_query regenerates it) and |Z|.
  batch_checks   expected results of the batch's histogram and predicate
                 queries by enumeration (oracle.hist / oracle.exists), for
                 every such query whose walk visits at most 3e8 prefixes
                 (a_1..a_{d-1}).  Lengths do not depend on the coordinate
                 order (permutation invariance is pinned on the oracle), so
                 each set is walked with its generators in descending order,
                 where the walk is shortest.  A histogram is kept as the
                 SHA-256 of its bins (little-endian u64, n / min g + 1 of
                 them) with its min and max length; a predicate as its verdict.

    python tests/golden/make_workloads.py batch_checks

recomputes only batch_checks (the rest of the file is kept).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fzinputs  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workloads.json")

BATCH_MASTER_SEED = 20240513
BATCH_QUERIES = 4096
BATCH_CAP = 10**8
SERVED_MASTER_SEED = 20240514
SERVED_QUERIES = 20000
STORE_CAP = 10**7


def single_small():
    w = fzinputs.single_small()
    n, g = w["n"], w["g"]
    h, lo, hi = oracle.hist(n, g)
    st = oracle.store(n, g)
    target = n // max(g) + 1
    return dict(n=n, g=g, count=oracle.dp_count(n, g), count_by_walk=oracle.count(n, g),
                min_len=lo, max_len=hi, nonzero_bins=int(np.count_nonzero(h)),
                exists_target=target, exists=oracle.exists(n, g, target),
                first=[int(x) for x in st[0]], last=[int(x) for x in st[-1]])


def single_large():
    n = 100000
    for seed in range(1000):
        g = fzinputs.single_large_generators(seed)
        c = oracle.dp_count(n, g)
        if 10**10 <= c <= 10**11:
            return dict(seed=seed, n=n, g=g, count=c, store_max_tuples=5 * 10**8)
    raise RuntimeError("no seed found")


def length_set():
    seed = 0
    g = fzinputs.length_set_generators(seed)
    series = oracle.dp_series(60000, g)
    idx = np.nonzero(series >= 10**11)[0]
    n = int(idx[0])
    return dict(seed=seed, n=n, g=g, count=int(series[n]), nbins=n // min(g) + 1)


def batch():
    seeds = fzinputs.query_seeds(BATCH_MASTER_SEED, BATCH_QUERIES)
    queries = []
    redraws = 0
    for s in seeds:
        rng = fzinputs.SplitMix64(s)
        while True:
            q = fzinputs.draw_query(rng)
            try:
                c = oracle.dp_count(q["n"], q["g"])
            except OverflowError:  # |Z| >= 2^64 - 1: far above the cap
                c = None
            if c is not None and c <= BATCH_CAP:
                break
            redraws += 1
        q["count"] = c
        queries.append(q)
    return dict(master_seed=BATCH_MASTER_SEED, cap=BATCH_CAP, redraws=redraws, queries=queries)


def served():
    seeds = fzinputs.query_seeds(SERVED_MASTER_SEED, SERVED_QUERIES)
    redraws, counts, modes = [], [], []
    for s in seeds:
        rng = fzinputs.SplitMix64(s)
        k = 0
        while True:
            q = fzinputs.draw_served(rng)
            cap = STORE_CAP if q["mode"] == "store" else BATCH_CAP
            try:
                c = oracle.dp_count(q["n"], q["g"])
            except OverflowError:
                c = None
            if c is not None and c <= cap:
                break
            k += 1
        redraws.append(k)
        counts.append(c)
        modes.append(q["mode"])
    return dict(master_seed=SERVED_MASTER_SEED, cap=BATCH_CAP, store_cap=STORE_CAP,
                store_share=fzinputs.STORE_SHARE, redraws=redraws, counts=counts,
                n_store=modes.count("store"))


BATCH_CHECK_MAX_PREFIXES = 3 * 10**8


def walk_prefixes(n, g):
    """Prefixes (a_1..a_{d-1}) with sum a_i g_i <= n: the nested loops' work."""
    return int(oracle.dp_series(n, g[:-1]).astype(np.float64).sum()) if len(g) > 1 else 1


def hist_digest(bins):
    return hashlib.sha256(np.ascontiguousarray(bins, dtype="<u8").tobytes()).hexdigest()


def batch_checks(queries):
    hists, preds = {}, {}
    for i, q in enumerate(queries):
        if q["mode"] not in ("hist", "exists"):
            continue
        n = q["n"]
        g = sorted(q["g"], reverse=True)
        if walk_prefixes(n, g) > BATCH_CHECK_MAX_PREFIXES:
            continue
        if q["mode"] == "hist":
            h, lo, hi = oracle.hist(n, g)
            assert int(h.sum()) == q["count"]
            hists[str(i)] = dict(nbins=len(h), sha256=hist_digest(h), min_len=lo, max_len=hi)
        else:
            preds[str(i)] = oracle.exists(n, g, q["target_len"])
    return dict(max_prefixes=BATCH_CHECK_MAX_PREFIXES, order="descending", hist=hists,
                exists=preds)


def main():
    t0 = time.time()
    if sys.argv[1:] == ["batch_checks"]:
        with open(OUT) as f:
            out = json.load(f)
        out["batch_checks"] = batch_checks(out["batch"]["queries"])
        with open(OUT, "w") as f:
            json.dump(out, f, separators=(",", ":"))
        print(f"updated batch_checks in {OUT} in {time.time() - t0:.1f}s")
        return
    b = batch()
    out = dict(
        note="written by tests/golden/make_workloads.py from the CPU oracle; do not edit",
        single_small=single_small(),
        single_large=single_large(),
        length_set=length_set(),
        batch=b,
        served=served(),
        batch_checks=batch_checks(b["queries"]),
    )
    with open(OUT, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(f"wrote {OUT} in {time.time() - t0:.1f}s")


if __name__ == "__main__":
    main()
