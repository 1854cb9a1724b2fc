"""GPU parity of the block walk's empty-row test (knob "empty_row_test"): a
block's rows whose remainder has no completion in the count table are
dropped before the block is walked.  Every consumer against the oracle with
the test on (the default with tables) and off, in both walk orders, with
slices cut at every modelled-work boundary (slices that begin and end inside
rows, some of them empty), with the trailing-index tables and with the
variant walk; on the benchmark set, the walker statistics: the same rows and
elements, fewer lane prefixes.  Also the slice cut with short last slices
(knob "short_last_slices") on and off."""
import numpy as np
import pytest

import fzinputs
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
        d = rng.randint(4, 8)
        g = [rng.randint(1, 12) for _ in range(d)]
        out.append((rng.randint(0, 60), g))
    return out


# Sets where whole rows are empty: the last three generators (caller order)
# or the three smallest (descending order) share a divisor that the row
# generator does not, so only one row in D has elements.
CASES = tiny_cases(7, 30) + [
    (3000, [108, 86, 164, 185, 145, 65]),      # last three share 5 (caller order)
    (4000, [73, 130, 222, 63, 57, 51]),        # three smallest share 3
    (2500, [41, 59, 77, 49, 35]),              # last three share 7
    (6000, [75, 10, 424, 529, 447, 983, 831, 750]),
    (10000, [11, 13, 17, 23]),
    (300, [3, 5, 7, 11, 13, 17, 19]),
    (12, [5, 5, 5, 1]),
    (4, [1] * 16),
]


def check_all(fz, n, g):
    want = oracle_store(n, g)
    assert fz.count(n, g) == len(want)
    assert fz.last_stats()["elements"] == len(want)
    h, lo, hi = fz.length_hist(n, g)
    oh, olo, ohi = oracle_hist(n, g)
    assert np.array_equal(h, oh) and (lo, hi) == (olo, ohi)
    for t in sorted({0, n // max(g) + 1, olo or 0, ohi or 0, (ohi or 0) + 1}):
        assert fz.exists(n, g, t) == oracle_exists(n, g, t)
    got, total = fz.enumerate_host(n, g, len(want) + 3)
    assert total == len(want)
    assert np.array_equal(got, want.reshape(-1, len(g)))


def with_knobs(fz, knobs, fn):
    try:
        for k, v in knobs.items():
            fz.config_set(k, v)
        fn()
    finally:
        for k in knobs:
            fz.config_set(k, 0)


@pytest.mark.parametrize("test", [0, 2], ids=["on", "off"])
@pytest.mark.parametrize("order", [0, 1], ids=["descending", "caller"])
def test_row_test_small_sets(fz, test, order):
    def run():
        for n, g in CASES:
            check_all(fz, n, g)
    with_knobs(fz, {"empty_row_test": test, "walk_order": order}, run)


@pytest.mark.parametrize("order", [0, 1], ids=["descending", "caller"])
def test_row_test_slices_inside_rows(fz, order):
    """One slice per unit of modelled work above 1: an empty row costs the
    skip weight, so slices begin and end inside rows, empty ones included."""
    def run():
        for n, g in CASES[-8:]:
            check_all(fz, n, g)
    with_knobs(fz, {"min_slice_work": 1, "walk_order": order}, run)


def test_row_test_with_trailing_tables(fz):
    """Count and store take full rows from the trailing tables; dropped rows
    take nothing."""
    def run():
        for n, g in CASES[-8:]:
            check_all(fz, n, g)
    with_knobs(fz, {"trailing": 1, "walk_order": 1}, run)


@pytest.mark.parametrize("order", [0, 1], ids=["descending", "caller"])
def test_row_test_with_variant_walk(fz, order):
    def run():
        for n, g in CASES[-8:]:
            check_all(fz, n, g)
    with_knobs(fz, {"variant": 1, "walk_order": order}, run)


def test_row_test_benchmark_statistics(fz):
    """The d = 6 count in the caller's order: four rows in five are empty
    (the last three generators share 5, the row generator does not).  With
    the test on, every row is still visited and every element counted, and
    only the non-empty rows' lane prefixes are walked."""
    big = GOLD["single_large"]
    stats = {}
    for test in (2, 0):
        def run():
            assert fz.count(big["n"], big["g"]) == big["count"]
            stats[test] = fz.last_stats()
        with_knobs(fz, {"empty_row_test": test, "walk_order": 1}, run)
    on, off = stats[0], stats[2]
    assert on["elements"] == off["elements"] == big["count"]
    assert on["rows"] == off["rows"]
    assert on["prefixes"] < 0.3 * off["prefixes"]


@pytest.mark.parametrize("short", [0, 2], ids=["short-last", "equal"])
def test_short_last_slices(fz, short):
    """Knob "short_last_slices": the last quarter of the slices is cut a
    quarter of the size of the others (or all equal); results are those of
    the oracle either way, with many slices per query (min_slice_work 1)."""
    def run():
        for n, g in CASES[-8:]:
            check_all(fz, n, g)
    with_knobs(fz, {"short_last_slices": short, "min_slice_work": 1}, run)
