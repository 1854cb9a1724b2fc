"""GPU parity of the single-query histogram's per-wave 32-bit bins (knobs
"wave_bins32", "wave_bins32_limit", "wave_bins32_copies"): each wave adds
its runs to 32-bit bins of its own in LDS (1, 2 or 4 interleaved copies,
lane l adding to copy l mod copies) and folds them, sign-extended, into the
workgroup's 64-bit bins before they could overflow.  Histograms against the
oracle with the 32-bit bins on and off, with each copy count, and with fold
thresholds small enough that waves fold after every few slices (and walk
slices above the threshold into the 64-bit bins directly)."""
import numpy as np
import pytest

import fzinputs
import oracle
from fzcheck import oracle_hist

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = fzinputs.load_golden()


@pytest.fixture(scope="module")
def fz():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2405_07989_amd as m
    return m


def cases():
    import random
    rng = random.Random(53)
    out = []
    for _ in range(30):
        d = rng.randint(1, 8)
        g = [rng.randint(1, 15) for _ in range(d)]
        out.append((rng.randint(0, 150 if d <= 3 else 70), g))
    return out + [
        (12, [5, 5, 5, 1]),
        (4, [1] * 16),
        (6000, [75, 10, 424, 529, 447, 983, 831, 750]),
        (3000, [13, 37, 38, 40, 41, 42]),
        (10000, [11, 13, 17, 23]),                 # 3.0e6 elements, 910 bins: the 64-bit set alone
        (2500, [11, 13, 17, 23]),                  # 227 bins
        (300, [3, 5, 7, 11, 13, 17, 19]),
    ]


@pytest.mark.parametrize("copies", [0, 1, 2, 4], ids=["copies-auto", "copies-1", "copies-2",
                                                     "copies-4"])
@pytest.mark.parametrize("on,limit", [(1, 0), (0, 0), (1, 1000), (1, 64), (1, 1)],
                         ids=["default", "off", "fold-1000", "fold-64", "fold-1"])
def test_histograms_with_wave_bins(fz, on, limit, copies):
    try:
        fz.config_set("wave_bins32", on)
        fz.config_set("wave_bins32_limit", limit)
        fz.config_set("wave_bins32_copies", copies)
        for n, g in cases():
            h, lo, hi = fz.length_hist(n, g)
            oh, olo, ohi = oracle_hist(n, g)
            assert np.array_equal(h, oh) and (lo, hi) == (olo, ohi), (n, g)
    finally:
        fz.config_set("wave_bins32", 1)
        fz.config_set("wave_bins32_limit", 0)
        fz.config_set("wave_bins32_copies", 0)


@pytest.mark.parametrize("copies", [0, 1, 2, 4], ids=["copies-auto", "copies-1", "copies-2",
                                                     "copies-4"])
@pytest.mark.parametrize("limit", [0, 4096], ids=["default", "fold-4096"])
def test_length_set_with_wave_bins(fz, limit, copies):
    """The d = 11 length set (271 bins, 1.0e11 elements)."""
    ls = GOLD["length_set"]
    try:
        fz.config_set("wave_bins32_limit", limit)
        fz.config_set("wave_bins32_copies", copies)
        h, lo, hi = fz.length_hist(ls["n"], ls["g"])
        want = oracle.dp_hist(ls["n"], ls["g"])
        assert np.array_equal(h, want) and int(h.sum()) == ls["count"]
        nz = np.nonzero(want)[0]
        assert (lo, hi) == (int(nz[0]), int(nz[-1]))
    finally:
        fz.config_set("wave_bins32_limit", 0)
        fz.config_set("wave_bins32_copies", 0)
