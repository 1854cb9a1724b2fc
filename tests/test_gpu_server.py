"""GPU tests of the request server (fz_server): queries submitted one at a
time, while others run, give exactly the results they give alone (single
batch) and the oracle's; admission refuses oversized queries; several client
threads may submit and wait at once."""
import random
import threading
import time

import numpy as np
import pytest

import fzinputs
import oracle
from fzcheck import check_against_oracle, tiny_queries

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fz():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2405_07989_amd as m
    return m


def with_outputs(qs, rows_of):
    for i, q in enumerate(qs):
        if q["mode"] == "store":
            rows = max(rows_of(i, q), 0)
            q["out"] = torch.zeros((max(rows, 1), len(q["g"])), dtype=torch.int32, device="cuda")
            q["max_tuples"] = rows
    return qs


def copy_query(q):
    c = {k: v for k, v in q.items() if k not in ("out", "_bins")}
    if q["mode"] == "store":
        c["out"] = torch.zeros_like(q["out"])
    return c


def same_result(q, a, qa, b, qb):
    assert a["status"] == b["status"], (q, a, b)
    if a["status"] < 0:
        return
    assert a["found"] == b["found"], q
    if not (q["mode"] == "exists" and a["found"]):
        assert a["count"] == b["count"], q
    if q["mode"] == "hist":
        assert np.array_equal(a["bins"], b["bins"]), q
        assert (a["min_len"], a["max_len"]) == (b["min_len"], b["max_len"])
    if q["mode"] == "store":
        assert a["written"] == b["written"] and a["total"] == b["total"], q
        w = a["written"]
        assert torch.equal(qa["out"][:w], qb["out"][:w]), q


@pytest.mark.parametrize("inflight,max_batch", [(1, 8), (3, 16), (8, 4096)])
def test_arrivals_match_the_oracle(fz, inflight, max_batch):
    rng = random.Random(inflight)
    qs = with_outputs(tiny_queries(10 + inflight, 150),
                      lambda i, q: oracle.dp_count(q["n"], q["g"]) + rng.randint(-2, 2))
    qs.append(dict(n=10, g=[3, 0], mode="count"))                    # invalid
    qs.append(dict(n=60, g=[5, 7, 2**24 + 1], mode="count"))         # last generator too large
    with fz.Server(max_inflight=inflight, max_batch=max_batch) as srv:
        tickets = []
        for i, q in enumerate(qs):
            tickets.append(srv.submit(q))
            if i % 7 == 0:
                time.sleep(rng.random() * 2e-4)
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert res[-2]["status"] == fz.FZ_EINVAL and res[-1]["status"] == fz.FZ_E2BIG
    for q, r in zip(qs[:-2], res[:-2]):
        check_against_oracle(q, r)
    assert st["submitted"] == st["completed"] == len(qs)
    assert st["launches"] >= 2 and 0 < st["p50_us"] <= st["p99_us"] <= st["max_us"]


def test_served_stream_alone_equals_mixed(fz):
    golden = fzinputs.load_golden()
    counts = golden["served"]["counts"]
    stream = fzinputs.served_stream(golden)[:600]
    cap = 200_000
    qs = with_outputs([dict(q) for q in stream], lambda i, q: min(counts[i], cap))
    alone_q = [copy_query(q) for q in qs]
    alone = [fz.batch([q])[0] for q in alone_q]
    gaps = fzinputs.exponential_gaps(7, 2000.0, len(qs))
    with fz.Server(max_inflight=4) as srv:
        tickets = []
        for q, gap in zip(qs, gaps):
            time.sleep(gap)
            tickets.append(srv.submit(q))
        mixed = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert st["launches"] > 1
    for i, (q, a, q_alone, b) in enumerate(zip(qs, mixed, alone_q, alone)):
        same_result(q, a, q, b, q_alone)
        assert a["status"] in (fz.FZ_OK, fz.FZ_TRUNCATED), (q, a)
        if q["mode"] in ("count", "hist"):
            assert a["count"] == counts[i]
        if q["mode"] == "store":
            assert a["total"] == counts[i] and a["written"] == min(counts[i], cap)


def test_admission(fz):
    n, g = 10000, [11, 13, 17, 23]            # |Z| = 3,009,519
    out = torch.zeros((1000, 4), dtype=torch.int32, device="cuda")
    small_out = torch.zeros((2000, 3), dtype=torch.int32, device="cuda")
    with fz.Server(max_store_tuples=1_000_000, mem_budget=1 << 22) as srv:
        big = srv.submit(dict(n=n, g=g, mode="store", out=out))
        small = srv.submit(dict(n=300, g=[3, 5, 7], mode="store", out=small_out))
        huge_tables = srv.submit(dict(n=900_000, g=[5, 7, 9, 11], mode="count"))
        fine = srv.submit(dict(n=n, g=g, mode="count"))
        r_big, r_small = srv.wait(big), srv.wait(small)
        r_huge, r_fine = srv.wait(huge_tables), srv.wait(fine)
    assert r_big["status"] == fz.FZ_E2BIG and r_big["total"] == 3009519
    assert r_huge["status"] == fz.FZ_E2BIG
    assert r_fine["status"] == 0 and r_fine["count"] == 3009519
    want = oracle.store(300, [3, 5, 7])
    assert r_small["status"] == 0 and r_small["written"] == len(want)
    assert np.array_equal(small_out[: len(want)].cpu().numpy().view(np.uint32), want)


def test_client_threads(fz):
    errors = []
    with fz.Server(max_inflight=2, max_batch=32) as srv:
        def client(seed):
            try:
                qs = [q for q in tiny_queries(seed, 60) if q["mode"] != "store"]
                ts = [srv.submit(q) for q in qs]
                for q, t in zip(qs, ts):
                    check_against_oracle(q, srv.wait(t))
            except Exception as e:  # noqa: BLE001 - reported below
                errors.append(e)
        th = [threading.Thread(target=client, args=(100 + i,)) for i in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=60)
        assert not any(t.is_alive() for t in th)
    assert not errors, errors[0]


def test_unknown_ticket(fz):
    with fz.Server() as srv:
        t = srv.submit(dict(n=100, g=[3, 5, 7], mode="count"))
        assert srv.wait(t)["count"] == oracle.count(100, [3, 5, 7])
        with pytest.raises(fz.FzError) as e:
            srv._live[t] = (dict(mode="count"), None)
            srv.wait(t)  # already collected
        assert e.value.status == fz.FZ_EINVAL
