"""Helpers shared by the GPU tests: seeded small queries and their check
against the CPU oracle.  The oracle's answers are memoized per query, so a
set that several tests check (every sparse set under every knob setting) is
walked on the CPU once per process; callers must not modify the arrays."""
import functools
import random

import numpy as np

import oracle


@functools.lru_cache(maxsize=None)
def _memo(kind, n, g, extra=None):
    g = list(g)
    if kind == "count":
        return oracle.count(n, g)
    if kind == "hist":
        return oracle.hist(n, g)
    if kind == "exists":
        return oracle.exists(n, g, extra)
    return oracle.store(n, g)


def oracle_count(n, g):
    return _memo("count", n, tuple(g))


def oracle_hist(n, g):
    return _memo("hist", n, tuple(g))


def oracle_exists(n, g, target):
    return _memo("exists", n, tuple(g), target)


def oracle_store(n, g):
    return _memo("store", n, tuple(g))


def tiny_queries(seed, count):
    rng = random.Random(seed)
    qs = []
    while len(qs) < count:
        d = rng.randint(1, 7)
        g = [rng.randint(1, 15) for _ in range(d)]
        n = rng.randint(0, 150 if d <= 3 else 70)
        if oracle.dp_count(n, g) > 200_000:
            continue
        mode = rng.choice(["count", "hist", "exists", "store"])
        q = dict(n=n, g=g, mode=mode)
        if mode == "exists":
            q["target_len"] = rng.randint(0, n // min(g) + 1)
        qs.append(q)
    return qs


def check_against_oracle(q, r):
    n, g = q["n"], q["g"]
    assert r["status"] >= 0, (q, r)
    if q["mode"] == "count":
        assert r["count"] == oracle_count(n, g)
    elif q["mode"] == "hist":
        h, lo, hi = oracle_hist(n, g)
        assert np.array_equal(r["bins"], h) and (r["min_len"], r["max_len"]) == (lo, hi)
        assert r["count"] == int(h.sum())
    elif q["mode"] == "exists":
        assert r["found"] == oracle_exists(n, g, q["target_len"])
    else:
        want = oracle_store(n, g)
        m = q.get("max_tuples", q["out"].shape[0])
        got = q["out"][: r["written"]].cpu().numpy().view(np.uint32)
        assert r["written"] == min(m, len(want)) and r["total"] == len(want)
        assert np.array_equal(got, want[: r["written"]])
