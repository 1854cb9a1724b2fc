"""The variant walk (knob "variant" = 1: the common-divisor skip over the last
two and three generators of Sec. 3.2.4 and closed-form run lengths) against
the oracle, bit-exact, for the consumers it serves (count, histogram,
predicate): tiny random sets, sets whose last generators share divisors (so
that lanes and rows are skipped), Table 1, the d=4 query, and the benchmark
queries (the d=6 count in both walk orders, the d=11 length-set histogram).
Stores keep the plain walk whatever the knob says, and are checked too."""
import random

import numpy as np
import pytest

import fzinputs
import oracle
from fzcheck import oracle_count, oracle_exists, oracle_hist, oracle_store

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fz():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2405_07989_amd as m
    m.config_set("variant", 1)
    yield m
    m.config_set("variant", 0)


def _check_all(fz, n, g):
    assert fz.count(n, g) == oracle_count(n, g), (n, g)
    h, lo, hi = fz.length_hist(n, g)
    oh, olo, ohi = oracle_hist(n, g)
    assert np.array_equal(h, oh) and (lo, hi) == (olo, ohi), (n, g)
    nb = len(oh)
    for t in {0, 1, n // max(g) + 1, (olo or 0), (ohi or 0), nb // 2, nb - 1}:
        assert fz.exists(n, g, t) == oracle_exists(n, g, t), (n, g, t)


def _divisor_sets(seed, count):
    """Sets whose last two or three generators share a divisor: lanes (x) and
    rows of the deepest row level are then strided."""
    rng = random.Random(seed)
    out = []
    while len(out) < count:
        d = rng.randint(4, 7)
        D3 = rng.choice([2, 3, 4, 5, 6])
        k = rng.choice([1, 2, 3])
        last3 = [D3 * rng.randint(1, 6) for _ in range(3)]
        last3[1] *= k  # a larger common divisor of the last two, sometimes
        last3[2] *= k
        g = [rng.randint(2, 20) for _ in range(d - 3)] + last3
        n = rng.randint(0, 400 if d <= 5 else 160)
        if oracle.dp_count(n, g) <= 300_000:
            out.append((n, g))
    return out


@pytest.mark.parametrize("order", [0, 1], ids=["descending", "caller"])
def test_variant_divisor_sets(fz, order):
    try:
        fz.config_set("walk_order", order)
        for n, g in _divisor_sets(5, 60):
            _check_all(fz, n, g)
    finally:
        fz.config_set("walk_order", 0)


@pytest.mark.parametrize("seed", [1, 2])
def test_variant_tiny_random(fz, seed):
    rng = random.Random(seed)
    for _ in range(80):
        d = rng.randint(1, 7)
        g = [rng.randint(1, 15) for _ in range(d)]
        n = rng.randint(0, 150 if d <= 3 else 70)
        _check_all(fz, n, g)


def test_variant_store_unchanged(fz):
    for n, g in [(300, [6, 10, 15, 12]), (10000, [11, 13, 17, 23]), (200, [4, 6, 9, 12, 18])]:
        want = oracle_store(n, g)
        out = torch.zeros((max(len(want), 1), len(g)), dtype=torch.int32, device="cuda")
        assert fz.enumerate_device(n, g, out) == (len(want), len(want))
        assert np.array_equal(out[: len(want)].cpu().numpy().view(np.uint32), want)


def test_variant_single_small(fz):
    s = fzinputs.load_golden()["single_small"]
    n, g = s["n"], s["g"]
    assert fz.count(n, g) == s["count"]
    h, lo, hi = fz.length_hist(n, g)
    assert np.array_equal(h, oracle.dp_hist(n, g)) and (lo, hi) == (s["min_len"], s["max_len"])
    assert not fz.exists(n, g, s["exists_target"]) and fz.exists(n, g, s["min_len"])


@pytest.mark.parametrize("order", [0, 1], ids=["descending", "drawn"])
def test_variant_large_count(fz, order):
    w = fzinputs.load_golden()["single_large"]
    try:
        fz.config_set("walk_order", order)
        assert fz.count(w["n"], w["g"]) == w["count"]
    finally:
        fz.config_set("walk_order", 0)


def test_variant_length_set_histogram(fz):
    ls = fzinputs.load_golden()["length_set"]
    h, lo, hi = fz.length_hist(ls["n"], ls["g"])
    assert int(h.sum()) == ls["count"]
    want = oracle.dp_hist(ls["n"], ls["g"])
    assert np.array_equal(h, want)
