"""Trailing-index tables (knob "trailing" = 1; Sec. 6.1, dynamic behavior):
a full row takes its elements Z(R, (g_{d-2}, g_{d-1}, g_d)) at once -- the
count from the count table, the store copied from a table of every Z(x).
Results against the oracle (count, rows element by element), truncated
stores that stop inside a copied row, and the d=6 query's 5e8-row store
against the plain walk's, word for word."""
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
    m.config_set("trailing", 1)
    yield m
    m.config_set("trailing", 0)


def _cases(seed, count):
    rng = random.Random(seed)
    out = []
    while len(out) < count:
        d = rng.randint(4, 7)
        g = [rng.randint(1, 15) for _ in range(d)]
        n = rng.randint(0, 80 if d <= 5 else 50)
        if oracle.dp_count(n, g) <= 200_000:
            out.append((n, g))
    return out


@pytest.mark.parametrize("order", [0, 1], ids=["descending", "caller"])
def test_trailing_count_and_store(fz, order):
    cases = _cases(11, 50) + [(10000, [11, 13, 17, 23]), (3000, [13, 37, 38, 40, 41])]
    try:
        fz.config_set("walk_order", order)
        for n, g in cases:
            want = oracle_store(n, g)
            assert fz.count(n, g) == len(want), (n, g)
            out = torch.zeros((max(len(want), 1), len(g)), dtype=torch.int32, device="cuda")
            assert fz.enumerate_device(n, g, out) == (len(want), len(want)), (n, g)
            assert np.array_equal(out[: len(want)].cpu().numpy().view(np.uint32), want), (n, g)
    finally:
        fz.config_set("walk_order", 0)


@pytest.mark.parametrize("m", [1, 63, 64, 65, 1000, 1234567])
def test_trailing_truncated_store(fz, m):
    n, g = 10000, [11, 13, 17, 23]
    want = oracle_store(n, g)
    out = torch.zeros((m, len(g)), dtype=torch.int32, device="cuda")
    total, written = fz.enumerate_device(n, g, out)
    assert total == len(want) and written == min(m, len(want))
    assert np.array_equal(out[:written].cpu().numpy().view(np.uint32), want[:written])


def test_trailing_large(fz):
    w = fzinputs.load_golden()["single_large"]
    n, g, M = w["n"], w["g"], w["store_max_tuples"]
    assert fz.count(n, g) == w["count"]
    got = torch.empty((M, len(g)), dtype=torch.int32, device="cuda")
    assert fz.enumerate_device(n, g, got) == (w["count"], M)
    fz.config_set("trailing", 0)
    try:
        want = torch.empty_like(got)
        assert fz.enumerate_device(n, g, want) == (w["count"], M)
        assert torch.equal(got, want)
    finally:
        fz.config_set("trailing", 1)
        del got
        torch.cuda.empty_cache()
