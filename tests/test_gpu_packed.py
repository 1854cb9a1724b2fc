"""GPU parity of the packed walk of short rows (knob "packed"): the lane
prefixes of up to 64 rows of the deepest row level are walked end to end,
64 at a time.  Every order-free consumer (count, length histogram,
predicate) against the oracle, with the walk forced on, forced off and
chosen by row length; with row skipping on and off; with slices cut at every
modelled-work boundary (knob "min_slice_work" = 1, so that most slices begin
and end inside a row); on the benchmark sets and at the size limit.  The
batch walker walks every order-free consumer packed, so the batch tests
cover it too."""
import numpy as np
import pytest

import fzinputs
import oracle
from fzcheck import oracle_exists, oracle_hist, oracle_store

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = fzinputs.load_golden()


@pytest.fixture(scope="module")
def fz():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2405_07989_amd as m
    return m


def tiny_cases(seed, count):
    import random
    rng = random.Random(seed)
    out = []
    for _ in range(count):
        d = rng.randint(4, 9)
        g = [rng.randint(1, 15) for _ in range(d)]
        out.append((rng.randint(0, 70), g))
    return out


CASES = tiny_cases(41, 40) + [
    (12, [5, 5, 5, 1]),                                   # repeats, last generator 1
    (4, [1] * 16),                                        # d = 16
    (25, [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53]),
    (6000, [75, 10, 424, 529, 447, 983, 831, 750]),       # sparse: most rows empty
    (5000, [5, 357, 149, 958, 122, 560, 756, 746]),
    (3000, [13, 37, 38, 40, 41, 42]),
    (10000, [11, 13, 17, 23]),                            # the d = 4 query
    (300, [3, 5, 7, 11, 13, 17, 19]),                     # dense, long rows
    # the last pair (two smallest) shares a divisor D that the third smallest
    # does not: lanes step x by D (common-divisor skip)
    (20000, [748, 647, 558, 525, 364, 26]),               # D = 26
    (5000, [101, 77, 30, 20]),                            # D = 10
    (3000, [97, 89, 45, 33, 22]),                         # D = 11
    (500, [15, 12, 8]),                                   # d = 3, D = 4
]


def check_order_free(fz, n, g):
    want = oracle_store(n, g)
    assert fz.count(n, g) == len(want)
    h, lo, hi = fz.length_hist(n, g)
    oh, olo, ohi = oracle_hist(n, g)
    assert np.array_equal(h, oh) and (lo, hi) == (olo, ohi)
    for t in sorted({0, n // max(g) + 1, olo or 0, ohi or 0, (ohi or 0) + 1}):
        assert fz.exists(n, g, t) == oracle_exists(n, g, t)


@pytest.mark.parametrize("skip", [0, 1, 2], ids=["auto", "skip", "noskip"])
@pytest.mark.parametrize("packed", [1, 2], ids=["packed", "plain"])
@pytest.mark.parametrize("order", [0, 1], ids=["descending", "caller"])
def test_packed_walk_small_sets(fz, packed, skip, order):
    try:
        fz.config_set("packed", packed)
        fz.config_set("skip_empty_rows", skip)
        fz.config_set("walk_order", order)
        for n, g in CASES:
            check_order_free(fz, n, g)
    finally:
        fz.config_set("packed", 0)
        fz.config_set("skip_empty_rows", 0)
        fz.config_set("walk_order", 0)


@pytest.mark.parametrize("skip", [1, 2], ids=["skip", "noskip"])
def test_packed_walk_slices_inside_rows(fz, skip):
    """One slice per unit of modelled work above 1: slices of a few
    elements, most of them starting and ending in the middle of a row."""
    try:
        fz.config_set("packed", 1)
        fz.config_set("skip_empty_rows", skip)
        fz.config_set("min_slice_work", 1)
        for n, g in CASES[-12:]:
            check_order_free(fz, n, g)
    finally:
        fz.config_set("packed", 0)
        fz.config_set("skip_empty_rows", 0)
        fz.config_set("min_slice_work", 0)


@pytest.mark.parametrize("packed", [0, 1, 2], ids=["auto", "packed", "plain"])
def test_packed_walk_benchmark_sets(fz, packed):
    """The d = 6 count and histogram and the d = 11 length set."""
    big, ls = GOLD["single_large"], GOLD["length_set"]
    try:
        fz.config_set("packed", packed)
        assert fz.count(big["n"], big["g"]) == big["count"]
        assert fz.last_stats()["elements"] == big["count"]
        h, lo, hi = fz.length_hist(big["n"], big["g"])
        assert np.array_equal(h, oracle.dp_hist(big["n"], big["g"]))
        h, lo, hi = fz.length_hist(ls["n"], ls["g"])
        want = oracle.dp_hist(ls["n"], ls["g"])
        assert np.array_equal(h, want) and int(h.sum()) == ls["count"]
        nz = np.nonzero(want)[0]
        assert (lo, hi) == (int(nz[0]), int(nz[-1]))
        assert fz.count(ls["n"], ls["g"]) == ls["count"]
    finally:
        fz.config_set("packed", 0)


def test_packed_walk_at_the_size_limit(fz):
    """d = 4 with n + 2 max g = 2^31 - 1: remainders up to 2^31, rows of
    hundreds of lane prefixes, 4092 elements (the oracle walks about 1e8
    prefixes)."""
    g = [2000003, 2700007, 3100019, 24011]
    n = 2**31 - 1 - 2 * max(g)
    want = oracle_store(n, g)
    lens = want.astype(np.int64).sum(axis=1)
    try:
        fz.config_set("packed", 1)
        assert fz.count(n, g) == len(want)
        h, lo, hi = fz.length_hist(n, g)
        assert (lo, hi) == (int(lens.min()), int(lens.max()))
        assert np.array_equal(h, np.bincount(lens, minlength=len(h)).astype(np.uint64))
        assert fz.exists(n, g, int(lens.min())) and fz.exists(n, g, int(lens.max()))
        assert not fz.exists(n, g, int(lens.max()) + 1)
    finally:
        fz.config_set("packed", 0)


def test_packed_walk_without_tables(fz):
    """The packed walk forced on a table-free walk (slices cut by splitWork,
    no count table: no row is dropped as empty, every row's prefixes are
    walked)."""
    try:
        fz.config_set("packed", 1)
        fz.config_set("tables", 2)
        for n, g in CASES:
            check_order_free(fz, n, g)
    finally:
        fz.config_set("packed", 0)
        fz.config_set("tables", 0)
