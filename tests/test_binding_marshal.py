"""The binding's batch marshalling (CPU): the fz_query array it builds holds
each query's fields, and a histogram query's bin count equals
fz_length_bins (at least 1) for valid and invalid inputs alike."""
import random

import paper_2405_07989_amd as fz


def test_histogram_bins_match_the_library():
    rng = random.Random(7)
    qs = []
    for _ in range(400):
        d = rng.randint(1, 17)
        g = [rng.choice([0, 1, rng.randint(1, 1000), rng.randint(1, 1 << 25)]) for _ in range(d)]
        # (valid ones stay small: their bins are allocated)
        n = rng.choice([0, rng.randint(0, 10**5), rng.randint(2**31, 2**31 + 10)])
        qs.append(dict(n=n, g=g, mode="hist"))
    qa, keep = fz._marshal(qs)
    for i, q in enumerate(qs):
        assert qa[i].nbins == max(fz.length_bins(q["n"], q["g"]), 1), q
        assert qa[i].n == q["n"] and qa[i].d == len(q["g"])
        assert [qa[i].g[k] for k in range(qa[i].d)] == q["g"]
        assert len(q["_bins"]) == qa[i].nbins


def test_fields_of_mixed_queries():
    qs = [dict(n=100, g=[3, 5, 7], mode="count"),
          dict(n=50, g=[2, 9], mode="exists", target_len=17),
          dict(n=70, g=[4, 6, 10, 15], mode="hist")]
    qa, keep = fz._marshal(qs)
    assert [qa[i].mode for i in range(3)] == [0, 2, 1]
    assert qa[1].target_len == 17 and qa[0].target_len == 0
    assert qa[2].nbins == 70 // 4 + 1 and qa[0].nbins == 0
