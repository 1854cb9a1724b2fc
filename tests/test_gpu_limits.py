"""GPU tests at the largest sizes the ABI accepts (include/fz.h: n + 2 max g
< 2^31; n < 2^30 when d <= 2; d <= 16), every consumer against the oracle's
enumeration.  The generators keep the oracle's walk short (about 1e8 prefixes
at most) while the count tables, remainders and histograms take their
largest sizes: the d = 3 set has 1.65e8 histogram bins and 6.4e9 table
entries."""
import numpy as np
import pytest

from fzcheck import oracle_store

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

G3 = [150001, 150011, 13]
N3 = 2**31 - 1 - 2 * max(G3)          # the largest n for these generators
G2 = [7, 11]
N2 = 2**30 - 1                        # the largest n with d = 2
G16 = list(range(2, 18))              # d = 16, the deepest walker
N16 = 100


@pytest.fixture(scope="module")
def fz():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2405_07989_amd as m
    return m


def check_all_consumers(fz, n, g):
    want = oracle_store(n, g)
    assert len(want) > 0
    assert fz.count(n, g) == len(want)
    got, total = fz.enumerate_host(n, g, len(want))
    assert total == len(want) and np.array_equal(got, want)
    lens = want.astype(np.int64).sum(axis=1)
    h, lo, hi = fz.length_hist(n, g)
    assert (lo, hi) == (int(lens.min()), int(lens.max()))
    assert np.array_equal(h, np.bincount(lens, minlength=len(h)).astype(np.uint64))
    assert fz.exists(n, g, int(lens.min())) and fz.exists(n, g, int(lens.max()))
    assert not fz.exists(n, g, int(lens.max()) + 1)
    ranks = np.array([0, 1, len(want) // 3, len(want) - 2, len(want) - 1])
    assert np.array_equal(fz.unrank(n, g, ranks), want[ranks])


def test_limit_n_plus_twice_the_largest_generator(fz):
    assert N3 + 2 * max(G3) == 2**31 - 1
    check_all_consumers(fz, N3, G3)


def test_limit_n_with_two_generators(fz):
    check_all_consumers(fz, N2, G2)


def test_limit_sixteen_generators(fz):
    check_all_consumers(fz, N16, G16)


def test_one_past_the_limits_is_refused(fz):
    with pytest.raises(fz.FzError) as e:
        fz.count(N3 + 1, G3)
    assert e.value.status == fz.FZ_EOVERFLOW
    with pytest.raises(fz.FzError) as e:
        fz.count(N2 + 1, G2)
    assert e.value.status == fz.FZ_EOVERFLOW
    with pytest.raises(fz.FzError) as e:
        fz.count(10, list(range(2, 19)))  # d = 17
    assert e.value.status == fz.FZ_EINVAL


def test_limit_n_in_a_batch(fz):
    # one query at the largest n (its count and work tables take 51 GB)
    want = oracle_store(N3, G3)
    want16 = oracle_store(N16, G16)
    lens16 = want16.astype(np.int64).sum(axis=1)
    qs = [dict(n=N3, g=G3, mode="count"),
          dict(n=N16, g=G16, mode="exists", target_len=int(lens16.max()) + 1),
          dict(n=N16, g=G16, mode="count"),
          dict(n=100, g=[3, 5, 7], mode="count")]
    res = fz.batch(qs)
    assert [r["status"] for r in res] == [0, 0, 0, 0]
    assert res[0]["count"] == len(want)
    assert not res[1]["found"] and res[1]["count"] == len(want16)
    assert res[2]["count"] == len(want16)
    assert res[3]["count"] == len(oracle_store(100, [3, 5, 7]))


@pytest.mark.parametrize("n,g", [(N3, G3), (N2, G2), (N16, G16)], ids=["d3", "d2", "d16"])
def test_limits_without_tables(fz, n, g):
    """The table-free walk (knob "tables" = 2: no count or work table, the
    slices cut by splitWork from the whole lexicographic range) at the size
    limits: count, histogram and predicate against the oracle's enumeration
    (stores always place rows by rank and keep their tables)."""
    want = oracle_store(n, g)
    lens = want.astype(np.int64).sum(axis=1)
    try:
        fz.config_set("tables", 2)
        assert fz.count(n, g) == len(want)
        h, lo, hi = fz.length_hist(n, g)
        assert (lo, hi) == (int(lens.min()), int(lens.max()))
        assert np.array_equal(h, np.bincount(lens, minlength=len(h)).astype(np.uint64))
        assert fz.exists(n, g, int(lens.min())) and fz.exists(n, g, int(lens.max()))
        assert not fz.exists(n, g, int(lens.max()) + 1)
    finally:
        fz.config_set("tables", 0)
