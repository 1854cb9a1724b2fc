"""The oracle's pins are strong enough to catch plausible mistakes.

Each case copies fz_oracle.c, plants one mistake (a dropped term, an
off-by-one bound, a wrong index, a transposed operand), builds the copy with
gcc in a temporary directory and runs a compact set of pins against it: brute
force, closed forms and the paper's candidate stream.  Every mutant must fail
at least one pin.  Nothing here touches the real oracle build.
"""
import itertools
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "fz_oracle.c")

MUTANTS = {
    "walk-loop-bound": ("for (uint64_t t = lo; t * gk <= rem; t++)",
                        "for (uint64_t t = lo; t * gk < rem; t++)"),
    "length-drops-last": ("for (uint32_t i = 0; i < w->d; i++) len += w->a[i];",
                          "for (uint32_t i = 0; i + 1 < w->d; i++) len += w->a[i];"),
    "start-path-sticky": ("walk_level(w, k + 1, rem - t * gk, on_start && t == lo);",
                          "walk_level(w, k + 1, rem - t * gk, on_start);"),
    "dp-count-skips-n": ("        for (uint64_t v = g[i]; v <= n; v++)\n            c[v] = sat_add(c[v], c[v - g[i]]);",
                         "        for (uint64_t v = g[i]; v < n; v++)\n            c[v] = sat_add(c[v], c[v - g[i]]);"),
    "dp-hist-wrong-length-index": ("c[(v - g[i]) * nbins + l - 1]", "c[(v - g[i]) * nbins + l]"),
    "unrank-wrong-level": ("uint64_t c = TT(k + 1, v - t * g[k]);", "uint64_t c = TT(k, v - t * g[k]);"),
    "first-candidate-floor": ("uint64_t x = (s->n + s->g[0] - 1) / s->g[0];",
                              "uint64_t x = s->n / s->g[0];"),
    "solve-no-round-up": ("a[pos + 1] = (residual + gnext - 1) / gnext;",
                          "a[pos + 1] = residual / gnext;"),
    "modulo-order-transposed": ("uint64_t order = s->g[d - 1] / gcd64(s->g[d - 2], s->g[d - 1]);",
                                "uint64_t order = s->g[d - 2] / gcd64(s->g[d - 2], s->g[d - 1]);"),
    "solve-wrong-generator": ("uint64_t gnext = s->g[pos + 1];", "uint64_t gnext = s->g[pos];"),
    "successor-keeps-tail": ("for (uint32_t j = pos + 1; j < d; j++) a[j] = 0;",
                             "for (uint32_t j = pos + 2; j < d; j++) a[j] = 0;"),
    "dp-series-skips-last": ("for (uint64_t v = g[i]; v <= nmax; v++)",
                             "for (uint64_t v = g[i]; v < nmax; v++)"),
    "dp-series-wrong-shift": ("series[v] = sat_add(series[v], series[v - g[i]]);",
                              "series[v] = sat_add(series[v], series[v - g[i] + 1]);"),
}


def brute(n, g):
    ranges = [range(n // gi + 1) for gi in g]
    return sorted(a for a in itertools.product(*ranges) if sum(x * y for x, y in zip(a, g)) == n)


CASES = [(37, [3, 5, 7]), (40, [4, 6, 9, 2]), (25, [2, 3]), (18, [5, 5, 3]), (30, [7]),
         (28, [1, 1, 1]), (0, [3, 4]), (45, [6, 10, 15]), (31, [4, 3, 2, 5])]


def run_pins():
    """A compact copy of the pins; raises on the first disagreement."""
    for n, g in CASES:
        ref = brute(n, g)
        assert [tuple(int(x) for x in r) for r in oracle.store(n, g)] == ref
        assert oracle.dp_count(n, g) == len(ref)
        nb = n // min(g) + 1
        h_ref = np.zeros(nb, dtype=np.uint64)
        for a in ref:
            h_ref[sum(a)] += 1
        assert np.array_equal(oracle.hist(n, g)[0], h_ref)
        assert np.array_equal(oracle.dp_hist(n, g), h_ref)
        for r, a in enumerate(ref):
            assert tuple(int(x) for x in oracle.unrank_dp(n, g, r)) == a
        for mod in (False, True):
            cs = oracle.candidate_stream(n, g, use_modulo=mod, cap=len(ref) + 1)
            assert [tuple(int(x) for x in r) for r in cs["valid"]] == ref[::-1]
        if ref:
            mid = list(ref[len(ref) // 2])
            got = oracle.store_from(n, g, mid, 3)
            assert [tuple(int(x) for x in r) for r in got] == ref[len(ref) // 2: len(ref) // 2 + 3]
    for d in (2, 3, 4):
        for n in (5, 12):
            assert oracle.dp_count(n, [1] * d) == math.comb(n + d - 1, d - 1)
    for g in ([3, 5, 7], [4, 6, 6], [2, 9]):
        s = oracle.dp_series(40, g)
        assert [int(x) for x in s] == [len(brute(v, g)) for v in range(41)]


def test_pins_pass_on_the_real_oracle():
    run_pins()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-shared", "-fPIC", "-o", str(lib), str(mutated)], check=True)
    with oracle.library(str(lib)):
        with pytest.raises((AssertionError, oracle.OracleError, OverflowError)):
            run_pins()
