"""Pins for the CPU oracle: each check ties it to something other than itself.

  * brute force over the box prod_i [0, n // g_i] on tiny inputs (pure Python),
  * closed forms: all-ones generators C(n+d-1, d-1); Popoviciu's formula for
    two coprime generators; [g | n] for one generator; n = 0,
  * the |Z(n)| column of the paper's Table 1 (Sec. 5.2),
  * structural facts: permutation invariance of counts and length histograms,
    a repeated generator multiplies the series by 1/(1 - x^g), two distinct
    generators give at most one element per length,
  * the paper's own candidate stream (Alg. 3.1, Sec. 3.2.4) against the
    nested-loop definition, Thm. 3.3's coordinate bound, and the partition
    by bounds of Sec. 4.

The oracle's two counting routes (enumeration and generating function) are
also checked against each other: they share no code.
"""
import itertools
import math
import os
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def brute(n, g):
    """All elements of Z(n, g) by exhaustive search of the box, sorted."""
    ranges = [range(n // gi + 1) for gi in g]
    sols = [a for a in itertools.product(*ranges) if sum(x * y for x, y in zip(a, g)) == n]
    return sorted(sols)


def tiny_cases(seed, count):
    rng = random.Random(seed)
    cases = []
    for _ in range(count):
        d = rng.randint(1, 5)
        g = [rng.randint(1, 12) for _ in range(d)]  # any order, repeats allowed
        n = rng.randint(0, 60 if d <= 3 else 40)
        cases.append((n, g))
    return cases


@pytest.mark.parametrize("n,g", tiny_cases(1, 150))
def test_walk_matches_brute_force(n, g):
    ref = brute(n, g)
    st = oracle.store(n, g)
    assert [tuple(int(x) for x in r) for r in st] == ref
    assert oracle.count(n, g) == len(ref)
    assert oracle.dp_count(n, g) == len(ref)
    nb = n // min(g) + 1
    h_ref = np.zeros(nb, dtype=np.uint64)
    for a in ref:
        h_ref[sum(a)] += 1
    h, lo, hi = oracle.hist(n, g)
    assert np.array_equal(h, h_ref)
    assert np.array_equal(oracle.dp_hist(n, g), h_ref)
    if ref:
        assert lo == min(sum(a) for a in ref) and hi == max(sum(a) for a in ref)
    else:
        assert lo is None and hi is None
    for target in range(nb + 1):
        assert oracle.exists(n, g, target) == any(sum(a) == target for a in ref)
    for r, a in enumerate(ref):
        assert tuple(int(x) for x in oracle.unrank_dp(n, g, r)) == a


@pytest.mark.parametrize("n,g", tiny_cases(2, 60))
def test_walk_from_start_tuple(n, g):
    ref = brute(n, g)
    rng = random.Random(n * 31 + len(g))
    for _ in range(5):
        # an arbitrary point of the box, not necessarily an element
        start = [rng.randint(0, n // gi + 1) for gi in g]
        idx = next((i for i, a in enumerate(ref) if list(a) >= start), len(ref))
        k = rng.randint(0, 6)
        got = oracle.store_from(n, g, start, k)
        assert [tuple(int(x) for x in r) for r in got] == ref[idx: idx + k]


@pytest.mark.parametrize("d", [1, 2, 3, 4, 6])
def test_all_ones_closed_form(d):
    for n in [0, 1, 2, 7, 30, 55]:
        want = math.comb(n + d - 1, d - 1)
        assert oracle.dp_count(n, [1] * d) == want
        assert oracle.count(n, [1] * d) == want
        h, lo, hi = oracle.hist(n, [1] * d)
        assert lo == hi == n and int(h[n]) == want and int(h.sum()) == want


@pytest.mark.parametrize("g", [[1], [3], [7], [10]])
def test_single_generator(g):
    for n in range(0, 80):
        want = 1 if n % g[0] == 0 else 0
        assert oracle.dp_count(n, g) == want
        assert oracle.count(n, g) == want


def popoviciu(n, a, b):
    """Number of nonnegative (x, y) with a x + b y = n for coprime a, b."""
    bp = pow(b, -1, a) if a > 1 else 0
    ap = pow(a, -1, b) if b > 1 else 0

    def frac(q):
        return q - math.floor(q)

    val = Fraction(n, a * b) - frac(Fraction(bp * n, a)) - frac(Fraction(ap * n, b)) + 1
    assert val.denominator == 1
    return int(val)


@pytest.mark.parametrize("a,b", [(2, 3), (3, 7), (5, 8), (11, 13), (17, 4), (1, 9)])
def test_two_generators_popoviciu(a, b):
    for n in list(range(0, 200)) + [1000, 4321, 99991]:
        want = popoviciu(n, a, b)
        assert oracle.dp_count(n, [a, b]) == want
        assert oracle.count(n, [a, b]) == want


def test_two_distinct_generators_one_element_per_length():
    for a, b in [(3, 5), (6, 4), (7, 2), (12, 18)]:
        for n in [0, 17, 60, 143, 500]:
            h, _, _ = oracle.hist(n, [a, b])
            assert int(h.max(initial=0)) <= 1


def test_zero_element():
    for g in [[4], [2, 3], [5, 5, 1], [9, 8, 7, 6]]:
        assert oracle.count(0, g) == 1
        st = oracle.store(0, g)
        assert st.shape == (1, len(g)) and not st.any()


@pytest.mark.parametrize("seed", range(6))
def test_permutation_invariance_and_repeats(seed):
    rng = random.Random(seed)
    g = [rng.randint(2, 30) for _ in range(rng.randint(2, 5))]
    n = rng.randint(100, 400)
    perm = g[:]
    rng.shuffle(perm)
    assert oracle.dp_count(n, g) == oracle.dp_count(n, perm) == oracle.count(n, perm)
    assert np.array_equal(oracle.dp_hist(n, g), oracle.dp_hist(n, perm))
    # a repeated generator h: |Z(n, g + [h])| = sum_t |Z(n - t h, g)|
    h = g[rng.randrange(len(g))]
    want = sum(oracle.dp_count(n - t * h, g) for t in range(n // h + 1))
    assert oracle.dp_count(n, g + [h]) == want == oracle.count(n, g + [h])


def load_table1():
    rows = []
    with open(os.path.join(HERE, "golden", "table1.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            gens, n, printed, status = line.split()
            g = [int(x) for x in gens.split(",")]
            exact = int(printed) + (int(status.split("+")[1]) if status.startswith("erratum") else 0)
            rows.append((g, int(n), int(printed), exact, status))
    return rows


TABLE1 = load_table1()


def test_table1_fixture_shape():
    assert len(TABLE1) == 29
    assert sum(1 for r in TABLE1 if r[4] == "printed") == 26


@pytest.mark.parametrize("g,n,printed,exact,status", TABLE1,
                         ids=[f"d{len(r[0])}-n{r[1]}" for r in TABLE1])
def test_table1_counts(g, n, printed, exact, status):
    assert oracle.dp_count(n, g) == exact
    if n * len(g) <= 200000 or len(g) <= 4:
        assert oracle.count(n, g) == exact


def test_table1_erratum_by_third_route():
    """(13,37,38,40,41,42), n=2000: printed 273456; count it with numpy over
    the first five coordinates, the sixth solved -- no oracle code involved."""
    g = [13, 37, 38, 40, 41, 42]
    n = 2000
    total = 0
    for a1 in range(n // g[0] + 1):
        r1 = n - a1 * g[0]
        for a2 in range(r1 // g[1] + 1):
            r2 = r1 - a2 * g[1]
            for a3 in range(r2 // g[2] + 1):
                r3 = r2 - a3 * g[2]
                a4 = np.arange(r3 // g[3] + 1)
                r4 = r3 - a4 * g[3]
                # for each a4, a5 runs over 0..r4//g4; a6 = rest/g5 must be integral
                for k in range(int(r4.max()) // g[4] + 1 if len(r4) else 0):
                    rest = r4 - k * g[4]
                    total += int(np.count_nonzero((rest >= 0) & (rest % g[5] == 0)))
    assert total == 273487 == 273456 + 31


@pytest.mark.parametrize("n,g", tiny_cases(3, 120))
@pytest.mark.parametrize("use_modulo", [False, True])
def test_candidate_stream_is_the_set_descending(n, g, use_modulo):
    """Alg. 3.1 (with or without the Sec. 3.2.4 skip), filtered by wasValid,
    lists Z in descending lex order; Thm. 3.3: a_i < n/g_i + 1 throughout."""
    ref = brute(n, g)
    cs = oracle.candidate_stream(n, g, use_modulo=use_modulo, cap=len(ref) + 1)
    got = [tuple(int(x) for x in r) for r in cs["valid"]]
    assert got == ref[::-1]
    assert cs["n_valid"] == len(ref)
    for i, gi in enumerate(g):
        assert cs["max_coord"][i] < Fraction(n, gi) + 1


def test_modulo_skip_reduces_candidates():
    for n, g in [(10000, [11, 13, 17, 23]), (3000, [13, 37, 38, 40, 41]), (5000, [13, 37, 38, 40])]:
        plain = oracle.candidate_stream(n, g, use_modulo=False, cap=0)
        mod = oracle.candidate_stream(n, g, use_modulo=True, cap=0)
        assert plain["n_valid"] == mod["n_valid"] == oracle.dp_count(n, g)
        assert mod["n_cand"] < plain["n_cand"]


@pytest.mark.parametrize("n,g", [(60, [3, 5, 7]), (45, [2, 9, 4, 6]), (100, [7, 3, 11]),
                                 (200, [13, 37, 38]), (90, [5, 5, 6, 2])])
def test_partition_by_bounds(n, g):
    """Sec. 4: with factorizations c_1 > c_2 > ... used as bounds, the worker
    that starts after c_k with bound c_{k+1} yields exactly the elements
    strictly between them; with the bounds themselves the slices cover Z once."""
    ref = brute(n, g)
    desc = ref[::-1]
    cuts = list(range(0, len(desc), 5))
    got = []
    for j, ci in enumerate(cuts):
        got.append(desc[ci])  # the split bound itself is saved by whoever made it
        nxt = cuts[j + 1] if j + 1 < len(cuts) else None
        bound = list(desc[nxt]) if nxt is not None else None
        cs = oracle.candidate_stream(n, g, start=list(desc[ci]), bound=bound, cap=len(ref) + 1)
        part = [tuple(int(x) for x in r) for r in cs["valid"]]
        assert part == desc[ci + 1: nxt]
        got.extend(part)
    assert got == desc


def test_single_small_workload_two_routes():
    n, g = 10000, [11, 13, 17, 23]
    assert oracle.count(n, g) == oracle.dp_count(n, g)
    h, lo, hi = oracle.hist(n, g)
    assert np.array_equal(h, oracle.dp_hist(n, g))
    st = oracle.store(n, g)
    assert (st.astype(np.int64) @ np.array(g, dtype=np.int64) == n).all()
    # strictly ascending lex order
    diff = st[1:].astype(np.int64) - st[:-1].astype(np.int64)
    first = np.argmax(diff != 0, axis=1)
    assert (diff[np.arange(len(diff)), first] > 0).all()
    rng = random.Random(7)
    for r in [0, 1, len(st) - 1] + [rng.randrange(len(st)) for _ in range(20)]:
        assert np.array_equal(oracle.unrank_dp(n, g, r), st[r])


@pytest.mark.parametrize("g", [[3, 5, 7], [4, 6, 6, 9], [2, 2, 3], [5], [7, 3],
                               [11, 13, 17, 23], [1, 1, 1, 1]])
def test_dp_series_against_walks_and_closed_forms(g):
    """fzo_dp_series (which chooses the length-set workload's n) pinned by
    routes that share none of its code: the single-n generating-function
    count for every v <= 3000, the nested-loop walk for every v <= 300 and
    every 37th v beyond (repeats included), brute force of the box on small
    v, and the closed forms C(v+d-1, d-1) (all ones), [g | v] (one
    generator) and Popoviciu (two coprime generators)."""
    vmax = 3000
    s = oracle.dp_series(vmax, g)
    assert len(s) == vmax + 1 and s.dtype == np.uint64
    for v in range(vmax + 1):
        assert int(s[v]) == oracle.dp_count(v, g), (v, g)
    for v in list(range(301)) + list(range(301, vmax + 1, 37)):
        if v <= (60 if min(g) == 1 and len(g) > 2 else 1200 if len(g) > 3 else vmax):
            assert int(s[v]) == oracle.count(v, g), (v, g)
    for v in range(0, 40):
        if math.prod(v // x + 1 for x in g) <= 20000:
            assert int(s[v]) == len(brute(v, g))
    if all(x == 1 for x in g):
        assert all(int(s[v]) == math.comb(v + len(g) - 1, len(g) - 1) for v in range(vmax + 1))
    if len(g) == 1:
        assert all(int(s[v]) == (v % g[0] == 0) for v in range(vmax + 1))
    if len(g) == 2 and math.gcd(*g) == 1:
        assert all(int(s[v]) == popoviciu(v, *g) for v in range(vmax + 1))


def test_dp_series_length_set_choice():
    """The length-set workload's n is the first v whose count reaches 1e11;
    the series there agrees with the independent single-n DP and with its
    neighbour, which must still be below 1e11 (the choice is the smallest)."""
    import json
    with open(os.path.join(HERE, "golden", "workloads.json")) as f:
        ls = json.load(f)["length_set"]
    n, g = ls["n"], ls["g"]
    s = oracle.dp_series(n, g)
    assert int(s[n]) == ls["count"] == oracle.dp_count(n, g) >= 10**11
    assert int(s.max(initial=0) if n == 0 else s[:n].max()) < 10**11
    assert oracle.dp_count(n - 1, g) == int(s[n - 1])


def test_dp_series_overflow_marker():
    # [x^v] 1/(1-x)^40 = C(v+39, 39) passes 2^64 - 1 near v = 160
    s = oracle.dp_series(300, [1] * 40)
    first = next(v for v in range(301) if math.comb(v + 39, 39) >= 2**64 - 1)
    assert all(int(s[v]) == math.comb(v + 39, 39) for v in range(first))
    assert all(int(s[v]) == 2**64 - 1 for v in range(first, 301))
