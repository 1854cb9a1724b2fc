"""GPU parity: every result of libfz against the CPU oracle, bit-exact.

All calls go through the C ABI (the ctypes binding).  Inputs are seeded; the
expected values come from the oracle at test time or from
tests/golden/workloads.json (written by the oracle).  Sizes:
  * tiny random inputs and every edge case the method has (empty set, one
    element, n = 0, d = 1 and 2, repeated generators, generators above n,
    the last generator 1, d = 16), checked element by element;
  * the d=4 single query (3,009,519 elements) in full, element by element;
  * Table 1's element / generator sets (counts);
  * the d=6 large query in the configuration the benchmark times: the count
    (3.2e10) against the oracle's generating-function count, and the 5e8-row
    store prefix by properties that pin it exactly (every row is an element,
    rows strictly ascend, the last row is the oracle's element of rank 5e8-1)
    plus windows compared row by row with the oracle;
  * the d=11 length-set query's histogram against the oracle's.
"""
import math
import os
import random

import numpy as np
import pytest

import fzinputs
import oracle
from fzcheck import oracle_store

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fz():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2405_07989_amd as m
    return m


GOLD = fzinputs.load_golden()


def rows(a):
    return [tuple(int(x) for x in r) for r in a]


def tiny_cases(seed, count, dmax=7):
    rng = random.Random(seed)
    out = []
    for _ in range(count):
        d = rng.randint(1, dmax)
        g = [rng.randint(1, 15) for _ in range(d)]
        n = rng.randint(0, 150 if d <= 3 else 70)
        out.append((n, g))
    return out


EDGE = [
    (1, [2, 4]),            # empty set
    (7, [2, 4, 6]),         # empty set, d = 3
    (0, [3, 5, 7]),         # n = 0: only the zero tuple
    (0, [4]),
    (9, [3]), (10, [3]),    # d = 1
    (17, [3, 5]), (1, [1, 1]),
    (12, [5, 5, 5, 1]),     # repeats, last generator 1
    (30, [100, 7, 3]),      # generator above n
    (23, [23, 23, 23]),
    (4, [1] * 16),          # d = 16 (the largest)
    (25, [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53]),
    (100, [7, 3, 1000000]),
    (5000, [4999, 1, 2]),
]


@pytest.mark.parametrize("n,g", tiny_cases(11, 60) + EDGE)
def test_small_inputs_all_consumers(fz, n, g):
    want = oracle_store(n, g)
    assert fz.count(n, g) == len(want)
    got, total = fz.enumerate_host(n, g, len(want) + 3)
    assert total == len(want)
    assert rows(got) == rows(want)
    h, lo, hi = fz.length_hist(n, g)
    oh, olo, ohi = oracle.hist(n, g)
    assert np.array_equal(h, oh) and lo == olo and hi == ohi
    for t in sorted({0, 1, n // max(g) + 1, olo or 0, ohi or 0, (ohi or 0) + 1}):
        assert fz.exists(n, g, t) == oracle.exists(n, g, t)
    if len(want):
        ranks = list(range(len(want)))
        assert rows(fz.unrank(n, g, ranks)) == rows(want)


# Sparse sets: most rows (a_1..a_{d-3}) have no element, and the walker skips
# empty subtrees by the count table.  Each is run with skipping automatic,
# forced on and forced off.
SPARSE = [
    (6000, [75, 10, 424, 529, 447, 983, 831, 750]),
    (9000, [94, 273, 587, 303, 743, 849, 336, 896]),
    (5000, [5, 357, 149, 958, 122, 560, 756, 746]),
    (12000, [733, 596, 429, 36, 995, 476, 741]),
    (3000, [13, 37, 38, 40, 41, 42]),
    (20000, [268, 422, 83, 155, 171, 995, 592, 886]),
]


@pytest.mark.parametrize("order", [0, 1], ids=["descending", "caller"])
@pytest.mark.parametrize("mode", [0, 1, 2], ids=["auto", "skip", "noskip"])
@pytest.mark.parametrize("n,g", SPARSE)
def test_sparse_sets_skip_empty_rows(fz, n, g, mode, order):
    want = oracle_store(n, g)
    try:
        fz.config_set("skip_empty_rows", mode)
        fz.config_set("walk_order", order)
        assert fz.count(n, g) == len(want)
        got, total = fz.enumerate_host(n, g, len(want))
        assert total == len(want) and np.array_equal(got, want)
        h, lo, hi = fz.length_hist(n, g)
        assert np.array_equal(h, oracle.dp_hist(n, g))
        lens = want.astype(np.int64).sum(axis=1)
        for t in (int(lens.min()), int(lens.max()), int(lens.min()) - 1, int(lens.max()) + 1):
            assert fz.exists(n, g, t) == bool((lens == t).any())
    finally:
        fz.config_set("skip_empty_rows", 0)
        fz.config_set("walk_order", 0)


@pytest.mark.parametrize("n,g", [c for c in tiny_cases(23, 80) + EDGE if len(c[1]) >= 4])
def test_small_inputs_forced_row_skipping(fz, n, g):
    want = oracle_store(n, g)
    try:
        fz.config_set("skip_empty_rows", 1)
        assert fz.count(n, g) == len(want)
        got, total = fz.enumerate_host(n, g, len(want) + 3)
        assert total == len(want) and rows(got) == rows(want)
        h, lo, hi = fz.length_hist(n, g)
        oh, olo, ohi = oracle.hist(n, g)
        assert np.array_equal(h, oh) and lo == olo and hi == ohi
    finally:
        fz.config_set("skip_empty_rows", 0)


# The pair table: each row's lanes take only the pair remainders that the
# last pair represents.  Forced on (and off) against the oracle.
@pytest.mark.parametrize("order", [0, 1], ids=["descending", "caller"])
@pytest.mark.parametrize("n,g", [c for c in tiny_cases(29, 40) + EDGE if len(c[1]) >= 4] + SPARSE)
def test_pair_table_all_consumers(fz, n, g, order):
    want = oracle_store(n, g)
    for mode in (1, 2):
        try:
            fz.config_set("pair_table", mode)
            fz.config_set("walk_order", order)
            assert fz.count(n, g) == len(want)
            got, total = fz.enumerate_host(n, g, len(want) + 3)
            assert total == len(want) and rows(got) == rows(want)
            h, lo, hi = fz.length_hist(n, g)
            assert np.array_equal(h, oracle.dp_hist(n, g))
            if len(want):
                lens = want.astype(np.int64).sum(axis=1)
                for t in (int(lens.min()), int(lens.max()) + 1):
                    assert fz.exists(n, g, t) == bool((lens == t).any())
        finally:
            fz.config_set("pair_table", 0)
            fz.config_set("walk_order", 0)


def test_unrank_rejects_rank_out_of_range(fz):
    with pytest.raises(fz.FzError) as e:
        fz.unrank(100, [3, 5, 7], [oracle.dp_count(100, [3, 5, 7])])
    assert e.value.status == fz.FZ_EINVAL


@pytest.fixture(scope="module")
def small(fz):
    w = GOLD["single_small"]
    return w["n"], w["g"], oracle.store(w["n"], w["g"])


def test_single_small_count_and_store(fz, small):
    n, g, want = small
    assert fz.count(n, g) == len(want) == GOLD["single_small"]["count"]
    got, total = fz.enumerate_host(n, g, len(want))
    assert total == len(want)
    assert np.array_equal(got, want)
    dev = torch.empty((len(want), len(g)), dtype=torch.int32, device="cuda")
    assert fz.enumerate_device(n, g, dev) == (len(want), len(want))
    assert np.array_equal(dev.cpu().numpy().view(np.uint32), want)


def test_single_small_hist_and_exists(fz, small):
    n, g, _ = small
    h, lo, hi = fz.length_hist(n, g)
    assert np.array_equal(h, oracle.dp_hist(n, g))
    oh, olo, ohi = oracle.hist(n, g)
    assert np.array_equal(h, oh) and (lo, hi) == (olo, ohi)
    tgt = GOLD["single_small"]["exists_target"]
    assert fz.exists(n, g, tgt) == oracle.exists(n, g, tgt) == GOLD["single_small"]["exists"]
    assert fz.exists(n, g, olo) and fz.exists(n, g, ohi)
    assert not fz.exists(n, g, ohi + 1)


@pytest.mark.parametrize("m", [0, 1, 2, 63, 64, 65, 1000, 123457, 3009518, 3009519, 3009600])
def test_single_small_truncated_store(fz, small, m):
    n, g, want = small
    cap = max(m, 1)
    got, total = fz.enumerate_host(n, g, m)
    assert total == len(want)
    assert np.array_equal(got, want[:m])


def test_single_small_unrank(fz, small):
    n, g, want = small
    rng = np.random.default_rng(5)
    ranks = np.concatenate([[0, 1, len(want) - 1], rng.integers(0, len(want), 5000)])
    assert np.array_equal(fz.unrank(n, g, ranks), want[ranks])


@pytest.mark.parametrize("knob,value", [("slices_per_wave", 1), ("slices_per_wave", 37),
                                        ("workgroups_per_cu", 1), ("workgroups_per_cu", 3),
                                        ("skip_empty_rows", 1), ("skip_empty_rows", 2),
                                        ("walk_order", 1)])
def test_tuning_knobs_do_not_change_results(fz, small, knob, value):
    n, g, want = small
    try:
        fz.config_set(knob, value)
        assert fz.count(n, g) == len(want)
        got, _ = fz.enumerate_host(n, g, len(want))
        assert np.array_equal(got, want)
        h, _, _ = fz.length_hist(n, g)
        assert np.array_equal(h, oracle.dp_hist(n, g))
    finally:
        fz.config_set(knob, 0)


TABLE1 = []
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1.txt")) as _f:
    for _line in _f:
        _line = _line.strip()
        if _line and not _line.startswith("#"):
            _gens, _n, _printed, _status = _line.split()
            TABLE1.append(([int(x) for x in _gens.split(",")], int(_n)))



# Histogram bins: one LDS set per workgroup up to 8191 bins (and a spare
# bin), global atomics beyond; both sides of that bound and of 2048 (the
# bound of per-wave bins), and a dense set whose runs collide in few bins
# across a workgroup's waves.
@pytest.mark.parametrize("n,g", [
    (6143, [3, 100, 101, 103]), (6144, [3, 100, 101, 103]),
    (24572, [3, 1000, 1001, 1003]),
    (24575, [3, 1000, 1001, 1003]), (24576, [3, 1000, 1001, 1003]),
    (30000, [5, 11, 13, 17]), (12000, [6, 11, 13, 17, 19]),
])
def test_histogram_bin_storage(fz, n, g):
    want = oracle.dp_hist(n, g)
    for order in (0, 1):
        try:
            fz.config_set("walk_order", order)
            h, lo, hi = fz.length_hist(n, g)
        finally:
            fz.config_set("walk_order", 0)
        assert len(h) == len(want) and np.array_equal(h, want), (n, g, order)
        nz = np.nonzero(want)[0]
        assert (lo, hi) == (int(nz[0]), int(nz[-1]))

@pytest.mark.parametrize("g,n", TABLE1, ids=[f"d{len(r[0])}-n{r[1]}" for r in TABLE1])
def test_table1_counts(fz, g, n):
    assert fz.count(n, g) == oracle.dp_count(n, g)


def test_length_set_histogram(fz):
    w = GOLD["length_set"]
    n, g = w["n"], w["g"]
    h, lo, hi = fz.length_hist(n, g)
    want = oracle.dp_hist(n, g)
    assert np.array_equal(h, want)
    assert int(h.sum()) == w["count"]
    nz = np.nonzero(want)[0]
    assert (lo, hi) == (int(nz[0]), int(nz[-1]))


def test_single_large_count(fz):
    w = GOLD["single_large"]
    assert fz.count(w["n"], w["g"]) == w["count"] == oracle.dp_count(w["n"], w["g"])
    st = fz.last_stats()
    assert st["elements"] == w["count"]


def test_single_large_unrank(fz):
    w = GOLD["single_large"]
    n, g = w["n"], w["g"]
    rng = random.Random(3)
    ranks = [0, 1, w["count"] - 1] + [rng.randrange(w["count"]) for _ in range(40)]
    got = fz.unrank(n, g, ranks)
    for r, row in zip(ranks, got):
        assert np.array_equal(row, oracle.unrank_dp(n, g, r))


def _check_ascending_valid(t, g, n, chunk=50_000_000):
    """Every row satisfies sum a_i g_i = n and rows strictly ascend (lex)."""
    gg = torch.tensor(g, dtype=torch.int64, device=t.device)
    N = t.shape[0]
    for s in range(0, N, chunk):
        e = min(N, s + chunk + 1)
        blk = t[s:e].to(torch.int64)
        assert bool(((blk * gg).sum(dim=1) == n).all())
        if blk.shape[0] > 1:
            dif = blk[1:] - blk[:-1]
            nz = dif != 0
            assert bool(nz.any(dim=1).all())
            first = nz.to(torch.int8).argmax(dim=1)
            assert bool((dif.gather(1, first[:, None]) > 0).all())
        del blk


def test_single_large_store_prefix(fz):
    """The benchmark's store run: the 5e8 lex-smallest elements of the d=6
    query, on the device."""
    w = GOLD["single_large"]
    n, g, M = w["n"], w["g"], w["store_max_tuples"]
    out = torch.empty((M, len(g)), dtype=torch.int32, device="cuda")
    total, written = fz.enumerate_device(n, g, out)
    assert (total, written) == (w["count"], M)
    _check_ascending_valid(out, g, n)
    assert np.array_equal(out[-1].cpu().numpy().view(np.uint32), oracle.unrank_dp(n, g, M - 1))
    head = oracle.store(n, g, 1_000_000)
    assert np.array_equal(out[:1_000_000].cpu().numpy().view(np.uint32), head)
    rng = random.Random(9)
    for p in [M - 1000] + [rng.randrange(M - 1000) for _ in range(12)]:
        start = oracle.unrank_dp(n, g, p)
        want = oracle.store_from(n, g, start, 1000)
        assert np.array_equal(out[p:p + 1000].cpu().numpy().view(np.uint32), want), p
    del out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("order", [0, 1], ids=["descending", "caller"])
def test_without_tables(fz, order):
    """The table-free walk (knob "tables" = 2): slices cut by splitWork with
    no count or work table, on tiny inputs, the edge cases, the sparse sets
    and the d=4 query, every order-free consumer against the oracle."""
    from fzcheck import check_against_oracle
    cases = tiny_cases(23, 60) + EDGE + SPARSE[:3] + [(10000, [11, 13, 17, 23])]
    try:
        fz.config_set("tables", 2)
        fz.config_set("walk_order", order)
        for n, g in cases:
            for mode in ("count", "hist", "exists"):
                q = dict(n=n, g=g, mode=mode, target_len=n // max(g) + 1)
                if mode == "count":
                    r = dict(status=0, count=fz.count(n, g))
                elif mode == "hist":
                    h, lo, hi = fz.length_hist(n, g)
                    r = dict(status=0, bins=h, min_len=lo, max_len=hi, count=int(h.sum()))
                else:
                    r = dict(status=0, found=fz.exists(n, g, q["target_len"]))
                check_against_oracle(q, r)
    finally:
        fz.config_set("tables", 0)
        fz.config_set("walk_order", 0)


def test_large_count_without_tables(fz):
    w = GOLD["single_large"]
    try:
        fz.config_set("tables", 2)
        assert fz.count(w["n"], w["g"]) == w["count"]
        ls = GOLD["length_set"]
        h, lo, hi = fz.length_hist(ls["n"], ls["g"])
        assert np.array_equal(h, oracle.dp_hist(ls["n"], ls["g"]))
    finally:
        fz.config_set("tables", 0)


@pytest.mark.parametrize("threads,share", [(4, 0), (4, 200000), (16, 0)])
def test_hybrid_pool(fz, threads, share):
    """Hybrid pool (knob "host_threads"): host threads walk the last slices of
    the work while the device walks the others; count, histogram and
    predicate against the oracle (share 0: the default share per thread;
    200000: a fifth of the work on the host)."""
    from fzcheck import check_against_oracle
    cases = tiny_cases(29, 40) + EDGE + SPARSE[:2] + [(10000, [11, 13, 17, 23])]
    try:
        fz.config_set("host_threads", threads)
        fz.config_set("host_share_ppm", share)
        for n, g in cases:
            for mode in ("count", "hist", "exists"):
                q = dict(n=n, g=g, mode=mode, target_len=n // max(g) + 1)
                if mode == "count":
                    r = dict(status=0, count=fz.count(n, g))
                elif mode == "hist":
                    h, lo, hi = fz.length_hist(n, g)
                    r = dict(status=0, bins=h, min_len=lo, max_len=hi, count=int(h.sum()))
                else:
                    r = dict(status=0, found=fz.exists(n, g, q["target_len"]))
                check_against_oracle(q, r)
        if threads == 16:
            w = GOLD["single_large"]
            assert fz.count(w["n"], w["g"]) == w["count"]
    finally:
        fz.config_set("host_threads", 0)
        fz.config_set("host_share_ppm", 0)
