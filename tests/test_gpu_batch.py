"""GPU parity of batches (fz_batch): many queries, mixed consumers, one launch.

Every query of a batch is checked against the CPU oracle (bit-exact), and a
query's result must be the same alone (the single-query entry points) and in
the mix.  The 4096-query workload (d in 3..8, generators in [5,1000], n
log-uniform in [1e3,1e6], count / histogram / predicate) is checked in full
against the oracle's generating-function counts, and its histograms and
predicates against the oracle bin by bin: by the oracle's bivariate
generating function where its table is small, and by the oracle's
enumeration (stored in tests/golden/workloads.json as a SHA-256 of the bins,
with min and max length, and as the predicate's verdict) for every query
whose enumeration is affordable, which covers each of the batch walker's
bin stores (64-bit LDS bins up to 1024, 32-bit LDS bins up to 2048, global
bins beyond).  The few largest are checked by the properties that hold at any
size: bins sum to |Z|; a predicate that found no witness visited all of Z.
"""
import hashlib
import random

import numpy as np
import pytest

import fzinputs
import oracle
from fzcheck import check_against_oracle, tiny_queries

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fz():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2405_07989_amd as m
    return m


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tiny_mixed_batch(fz, seed):
    qs = tiny_queries(seed, 120)
    for q in qs:
        if q["mode"] == "store":
            cnt = oracle.dp_count(q["n"], q["g"])
            rows = max(cnt + random.Random(q["n"]).randint(-2, 2), 1)
            q["out"] = torch.zeros((rows, len(q["g"])), dtype=torch.int32, device="cuda")
    res = fz.batch(qs)
    for q, r in zip(qs, res):
        check_against_oracle(q, r)


def test_invalid_queries_do_not_stop_the_batch(fz):
    qs = [dict(n=100, g=[3, 5, 7], mode="count"),
          dict(n=100, g=[3, 0, 7], mode="count"),          # g_i = 0
          dict(n=2**31, g=[3, 5], mode="count"),          # too large
          dict(n=50, g=[4, 6], mode="hist"),
          dict(n=60, g=[5, 7, 2**24 + 1], mode="count"),   # last generator too large
          dict(n=77, g=[2, 9, 11, 4], mode="exists", target_len=20)]
    res = fz.batch(qs)
    assert res[1]["status"] == fz.FZ_EINVAL
    assert res[2]["status"] == fz.FZ_EOVERFLOW
    assert res[4]["status"] == fz.FZ_E2BIG
    for i in (0, 3, 5):
        check_against_oracle(qs[i], res[i])


def test_empty_batch(fz):
    assert fz.batch([]) == []


def test_store_queries_in_a_batch(fz):
    qs = []
    for n, g, m in [(10000, [11, 13, 17, 23], 3009519), (10000, [11, 13, 17, 23], 1000),
                    (5000, [13, 37, 38, 40], 10**6), (3000, [13, 37, 38, 40, 41], 50000),
                    (1, [2, 4], 5)]:
        qs.append(dict(n=n, g=g, mode="store", max_tuples=m,
                       out=torch.zeros((m, len(g)), dtype=torch.int32, device="cuda")))
    qs.append(dict(n=10000, g=[11, 13, 17, 23], mode="count"))
    res = fz.batch(qs)
    for q, r in zip(qs, res):
        check_against_oracle(q, r)
    assert res[1]["status"] == fz.FZ_TRUNCATED


@pytest.fixture(scope="module")
def workload():
    return fzinputs.load_golden()["batch"]["queries"]


@pytest.fixture(scope="module")
def batch_result(fz, workload):
    qs = [dict(n=q["n"], g=q["g"], mode=q["mode"], target_len=q["target_len"]) for q in workload]
    return qs, fz.batch(qs)


def test_workload_counts(batch_result, workload):
    qs, res = batch_result
    for q, r, w in zip(qs, res, workload):
        assert r["status"] == 0, (q, r)
        if q["mode"] in ("count", "hist"):
            assert r["count"] == w["count"], q
        if q["mode"] == "hist":
            assert int(r["bins"].sum()) == w["count"]
        if q["mode"] == "exists" and not r["found"]:
            assert r["count"] == w["count"], q  # no witness: all of Z was visited


def test_workload_histograms_and_predicates(batch_result, workload):
    qs, res = batch_result
    checked_h = checked_e = 0
    for q, r, w in zip(qs, res, workload):
        nb = q["n"] // min(q["g"]) + 1
        if (q["n"] + 1) * nb > 3_000_000:
            continue
        if q["mode"] == "hist":
            assert np.array_equal(r["bins"], oracle.dp_hist(q["n"], q["g"])), q
            checked_h += 1
        elif q["mode"] == "exists":
            t = q["target_len"]
            want = t < nb and bool(oracle.dp_hist(q["n"], q["g"])[t] > 0)
            assert r["found"] == want, q
            checked_e += 1
    assert checked_h > 200 and checked_e > 200


def _bin_store(nbins):
    """The batch walker's store for a histogram of nbins bins (the rule of
    fz_batch): 64-bit LDS bins up to 1024, 32-bit LDS bins up to 2048 (every
    workload query has fewer than 2^30 elements), global bins beyond."""
    return "lds64" if nbins <= 1024 else "lds32" if nbins <= 2048 else "global"


def test_workload_against_oracle_enumeration(batch_result, workload):
    """Bin by bin against the oracle's enumeration (tests/golden), on every
    bin store, and predicates that found a witness against the oracle's
    verdict."""
    qs, res = batch_result
    checks = fzinputs.load_golden()["batch_checks"]
    per_store = {"lds64": 0, "lds32": 0, "global": 0}
    big64 = found = 0
    for key, want in checks["hist"].items():
        i = int(key)
        q, r = qs[i], res[i]
        assert q["mode"] == "hist" and r["status"] == 0
        assert len(r["bins"]) == want["nbins"], q
        got = hashlib.sha256(np.ascontiguousarray(r["bins"], dtype="<u8").tobytes()).hexdigest()
        assert got == want["sha256"], (i, q)
        assert (r["min_len"], r["max_len"]) == (want["min_len"], want["max_len"]), (i, q)
        per_store[_bin_store(want["nbins"])] += 1
        big64 += want["nbins"] <= 1024 and (q["n"] + 1) * want["nbins"] > 3_000_000
    for key, want in checks["exists"].items():
        i = int(key)
        assert qs[i]["mode"] == "exists" and res[i]["status"] == 0
        assert res[i]["found"] == want, (i, qs[i])
        found += want
    assert per_store["lds32"] >= 20 and per_store["global"] >= 20 and big64 >= 20, per_store
    assert found >= 50


# Batch bin stores on both sides of 1024 bins (64-bit LDS bins), 2048 (32-bit
# LDS bins) and beyond (global atomics); dense sets whose runs pile up in few
# bins, so that 32-bit bins go negative between flushes.
BIN_EDGES = [(3069, [3, 100, 101, 103]), (3072, [3, 100, 101, 103]),
             (6141, [3, 100, 101, 103]), (6144, [3, 100, 101, 103]),
             (10235, [5, 11, 13, 17]), (5115, [5, 11, 13, 17]), (5120, [5, 11, 13, 17]),
             (10240, [5, 11, 13, 17]), (12281, [6, 11, 13, 17, 19])]


@pytest.mark.parametrize("order", [0, 1], ids=["descending", "caller"])
def test_batch_histogram_bin_stores(fz, order):
    qs = [dict(n=n, g=g, mode="hist") for n, g in BIN_EDGES]
    # the same queries again beside a large one, which changes the cut
    qs += [dict(n=100000, g=[108, 86, 164, 185, 145, 65], mode="count")] + \
          [dict(n=n, g=g, mode="hist") for n, g in BIN_EDGES]
    assert {_bin_store(n // min(g) + 1) for n, g in BIN_EDGES} == {"lds64", "lds32", "global"}
    try:
        fz.config_set("walk_order", order)
        res = fz.batch(qs)
    finally:
        fz.config_set("walk_order", 0)
    for q, r in zip(qs, res):
        assert r["status"] == 0, q
        if q["mode"] != "hist":
            continue
        want = oracle.dp_hist(q["n"], q["g"])
        assert len(r["bins"]) == len(want) and np.array_equal(r["bins"], want), (q, order)
        nz = np.nonzero(want)[0]
        assert (r["min_len"], r["max_len"]) == (int(nz[0]), int(nz[-1]))


def test_alone_equals_in_the_mix(fz, batch_result, workload):
    qs, res = batch_result
    rng = random.Random(4)
    for i in rng.sample(range(len(qs)), 60):
        q, r = qs[i], res[i]
        if q["mode"] == "count":
            assert fz.count(q["n"], q["g"]) == r["count"]
        elif q["mode"] == "hist":
            h, lo, hi = fz.length_hist(q["n"], q["g"])
            assert np.array_equal(h, r["bins"]) and (lo, hi) == (r["min_len"], r["max_len"])
        else:
            assert fz.exists(q["n"], q["g"], q["target_len"]) == r["found"]


def test_autotune_keeps_results(fz):
    qs = [q for q in tiny_queries(5, 80) if q["mode"] != "store"]
    before = fz.batch(qs)
    try:
        t = fz.autotune(qs, reps=1)
        assert t["candidates"] == 15 and t["ms"] <= t["default_ms"]
        assert t["slices_per_wave"] in (4, 8, 16, 32, 64) and t["workgroups_per_cu"] in (2, 4, 8)
        after = fz.batch(qs)
    finally:
        fz.config_set("slices_per_wave", 0)
        fz.config_set("workgroups_per_cu", 0)
    for q, a, b in zip(qs, before, after):
        assert a["status"] == b["status"] == 0 and a["found"] == b["found"], q
        # a predicate that found a witness stops early: how many elements it
        # visited first depends on the slicing
        if not (q["mode"] == "exists" and a["found"]):
            assert a["count"] == b["count"], q
        if q["mode"] == "hist":
            assert np.array_equal(a["bins"], b["bins"])


@pytest.mark.parametrize("order", [0, 1], ids=["descending", "caller"])
@pytest.mark.parametrize("mode", [0, 1, 2], ids=["auto", "skip", "noskip"])
def test_row_skipping_in_a_batch(fz, mode, order):
    from test_gpu_parity import SPARSE
    qs = []
    for n, g in SPARSE:
        for m in ("count", "hist", "exists", "store"):
            q = dict(n=n, g=g, mode=m, target_len=n // max(g) + 1)
            if m == "store":
                q["out"] = torch.zeros((oracle.dp_count(n, g), len(g)), dtype=torch.int32,
                                       device="cuda")
            qs.append(q)
    qs += [q for q in tiny_queries(31, 60) if q["mode"] != "store"]
    try:
        fz.config_set("skip_empty_rows", mode)
        fz.config_set("walk_order", order)
        res = fz.batch(qs)
    finally:
        fz.config_set("skip_empty_rows", 0)
        fz.config_set("walk_order", 0)
    for q, r in zip(qs, res):
        check_against_oracle(q, r)


def test_batch_graph_replays_match_plain_launches(fz):
    """Phase 2 of a batch runs as a HIP graph updated in place from batch to
    batch; several batches of different shapes, each run with the graph and
    with plain launches, eager single-query work in between."""
    w = fzinputs.load_golden()["batch"]["queries"]
    groups = [w[:200], w[1000:1100], tiny_queries(41, 80), w[2000:2600], w[:200]]
    for r, group in enumerate(groups):
        qs = [dict(n=q["n"], g=q["g"], mode=q["mode"],
                   target_len=q.get("target_len", 0)) for q in group if q["mode"] != "store"]
        try:
            fz.config_set("batch_graph", 1)
            got = fz.batch([dict(q) for q in qs])
            fz.config_set("batch_graph", 0)
            want = fz.batch([dict(q) for q in qs])
        finally:
            fz.config_set("batch_graph", 1)
        assert fz.count(10000, [11, 13, 17, 23]) == 3009519  # eager work between replays
        for q, a, b in zip(qs, got, want):
            assert a["status"] == b["status"] == 0, (r, q)
            assert a["found"] == b["found"], (r, q)
            if not (q["mode"] == "exists" and a["found"]):
                assert a["count"] == b["count"], (r, q)
            if q["mode"] == "hist":
                assert np.array_equal(a["bins"], b["bins"]), (r, q)


@pytest.mark.parametrize("order", [0, 1], ids=["descending", "caller"])
def test_sparse_pairs_in_a_batch(fz, order):
    # Sparse last pairs, which single queries walk by the pair table; a batch
    # walks them without it, whatever the knob says, and must agree with the
    # oracle either way.
    from test_gpu_parity import SPARSE
    qs = []
    for n, g in SPARSE:
        for m in ("count", "hist", "exists", "store"):
            q = dict(n=n, g=g, mode=m, target_len=n // max(g) + 1)
            if m == "store":
                q["out"] = torch.zeros((oracle.dp_count(n, g), len(g)), dtype=torch.int32,
                                       device="cuda")
            qs.append(q)
    qs += [q for q in tiny_queries(37, 60) if q["mode"] != "store"]
    try:
        fz.config_set("pair_table", 1)
        fz.config_set("walk_order", order)
        res = fz.batch(qs)
    finally:
        fz.config_set("pair_table", 0)
        fz.config_set("walk_order", 0)
    for q, r in zip(qs, res):
        check_against_oracle(q, r)


def test_large_queries_in_a_small_batch(fz, batch_result, workload):
    """A batch of a few queries with large tables (n + 1 > 2^16 entries per
    row) builds them row by row, each row shared by several workgroups; every
    result must equal the same query's in the 4096-query batch (one workgroup
    per query) and its stored count."""
    qs, res = batch_result
    idx = [i for i, q in enumerate(qs) if q["n"] + 1 > 1 << 16][:48]
    assert len(idx) == 48
    sub = [dict(qs[i]) for i in idx]
    small = fz.batch(sub)
    for i, r in zip(idx, small):
        big, w = res[i], workload[i]
        assert r["status"] == 0 and big["status"] == 0
        if qs[i]["mode"] in ("count", "hist"):
            assert r["count"] == big["count"] == w["count"], qs[i]
        if qs[i]["mode"] == "hist":
            assert np.array_equal(r["bins"], big["bins"]), qs[i]
            assert (r["min_len"], r["max_len"]) == (big["min_len"], big["max_len"])
        if qs[i]["mode"] == "exists":
            assert r["found"] == big["found"], qs[i]
