"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This module draws generator sets, elements and query mixes; it holds none of
the enumeration arithmetic (no counting, no factorizations).  Anything that
needs a count (for example the cap that rejects queries whose factorization set
is too large, or the element n whose set has about 1e11 elements) is decided
once by ``tests/golden/make_workloads.py`` with the CPU oracle and stored in
``tests/golden/workloads.json``.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), the 64-bit finaliser variant
published with it: state += 0x9E3779B97F4A7C15, then two xor-shift-multiply
rounds and a final xor-shift.
"""
from __future__ import annotations

import json
import math
import os

MASK64 = (1 << 64) - 1

GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "tests", "golden", "workloads.json")


class SplitMix64:
    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform_int(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] by rejection (no modulo bias)."""
        span = hi - lo + 1
        limit = (1 << 64) - ((1 << 64) % span)
        while True:
            x = self.next()
            if x < limit:
                return lo + x % span

    def uniform01(self) -> float:
        """Uniform double in [0, 1) from the top 53 bits."""
        return (self.next() >> 11) * (1.0 / (1 << 53))


def draw_distinct(rng: SplitMix64, k: int, lo: int, hi: int) -> list[int]:
    """k distinct integers uniform in [lo, hi], in drawn order, whose gcd is 1;
    the whole set is drawn again when the gcd is larger."""
    while True:
        out: list[int] = []
        while len(out) < k:
            x = rng.uniform_int(lo, hi)
            if x not in out:
                out.append(x)
        g = 0
        for x in out:
            g = math.gcd(g, x)
        if g == 1:
            return out


# --- the five workloads ----------------------------------------------------

def single_small():
    """d=4 generators (11,13,17,23), n=10000."""
    return dict(n=10000, g=[11, 13, 17, 23])


def single_large_generators(seed: int) -> list[int]:
    """d=6 distinct generators uniform in [20,200], gcd 1, drawn order."""
    return draw_distinct(SplitMix64(seed), 6, 20, 200)


def length_set_generators(seed: int) -> list[int]:
    """d=10 distinct generators uniform in [50,500] with gcd 1, followed by a
    copy of one of them (chosen by the same stream), 11 entries in all."""
    rng = SplitMix64(seed)
    g = draw_distinct(rng, 10, 50, 500)
    g.append(g[rng.uniform_int(0, 9)])
    return g


MODES = ("count", "hist", "exists")


def draw_query(rng: SplitMix64) -> dict:
    """One mixed-batch query: d uniform in {3..8}, distinct generators uniform
    in [5,1000] with gcd 1, n log-uniform in [1e3,1e6], consumer uniform among
    count / hist / exists; the predicate's target length is floor(n/max g)+1."""
    d = rng.uniform_int(3, 8)
    g = draw_distinct(rng, d, 5, 1000)
    n = int(round(10.0 ** (3.0 + 3.0 * rng.uniform01())))
    mode = MODES[rng.uniform_int(0, 2)]
    return dict(n=n, g=g, mode=mode, target_len=n // max(g) + 1)


STORE_SHARE = 0.2


def draw_served(rng: SplitMix64) -> dict:
    """One query of the served stream: drawn as draw_query, then made a store
    query with probability STORE_SHARE (one more uniform draw)."""
    q = draw_query(rng)
    if rng.uniform01() < STORE_SHARE:
        q["mode"] = "store"
    return q


def served_query(seed: int, redraws: int) -> dict:
    """Query of the served stream with this seed, after the recorded number
    of redraws (draws rejected for their size when the stream was fixed)."""
    rng = SplitMix64(seed)
    for _ in range(redraws + 1):
        q = draw_served(rng)
    return q


def query_seed(master_seed: int, i: int) -> int:
    """Seed of query i: the i-th output of SplitMix64(master_seed)."""
    rng = SplitMix64(master_seed)
    x = 0
    for _ in range(i + 1):
        x = rng.next()
    return x


def query_seeds(master_seed: int, count: int) -> list[int]:
    rng = SplitMix64(master_seed)
    return [rng.next() for _ in range(count)]


def exponential_gaps(seed: int, rate_qps: float, count: int) -> list[float]:
    """Poisson arrivals: inter-arrival gaps in seconds, -ln(1-U)/rate."""
    rng = SplitMix64(seed)
    return [-math.log(1.0 - rng.uniform01()) / rate_qps for _ in range(count)]


def load_golden() -> dict:
    """The stored choices and expected values (see module docstring)."""
    with open(GOLDEN) as f:
        return json.load(f)


def served_stream(golden: dict | None = None) -> list[dict]:
    """The served stream's queries, in arrival order, from the stored seeds."""
    w = (golden or load_golden())["served"]
    seeds = query_seeds(w["master_seed"], len(w["redraws"]))
    return [served_query(s, k) for s, k in zip(seeds, w["redraws"])]
