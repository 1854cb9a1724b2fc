"""GPU tests of ordering with the caller's torch work: an output tensor that
torch is still filling when the library is called must not be written before
the fill ends (the binding queues the library's work after torch's current
stream).  A fill that landed after the walker would leave zero rows, which
are not elements of Z(n, g) for n > 0."""
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# 200,062,341 rows x 6 columns: a 4.8 GB fill, long enough to overlap the
# library's first kernels if nothing orders them.
N, G = 12265, [7, 11, 13, 17, 997, 1009]
ROWS = 200_062_341


@pytest.fixture(scope="module")
def fz():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2405_07989_amd as m
    return m


def all_elements(out, n, g):
    gt = torch.tensor(g, dtype=torch.int32, device=out.device)
    return bool(((out * gt).sum(dim=1) == n).all().item())


def test_row_count_is_the_oracles():
    assert oracle.dp_count(N, G) == ROWS


def test_store_after_a_fill_on_the_default_stream(fz):
    out = torch.full((ROWS, len(G)), 0, dtype=torch.int32, device="cuda")
    total, written = fz.enumerate_device(N, G, out)
    assert total == written == ROWS
    assert all_elements(out, N, G)
    del out


def test_store_after_a_fill_on_a_side_stream(fz):
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = torch.zeros((ROWS, len(G)), dtype=torch.int32, device="cuda")
        total, written = fz.enumerate_device(N, G, out)
    torch.cuda.current_stream().wait_stream(s)
    assert total == written == ROWS
    assert all_elements(out, N, G)
    del out


def test_batch_store_after_a_fill(fz):
    out = torch.zeros((ROWS, len(G)), dtype=torch.int32, device="cuda")
    small = torch.zeros((oracle.dp_count(300, [3, 5, 7]), 3), dtype=torch.int32, device="cuda")
    res = fz.batch([dict(n=N, g=G, mode="store", out=out),
                    dict(n=300, g=[3, 5, 7], mode="store", out=small),
                    dict(n=N, g=G, mode="count")])
    assert [r["status"] for r in res] == [0, 0, 0]
    assert res[0]["written"] == ROWS and res[2]["count"] == ROWS
    assert all_elements(out, N, G) and all_elements(small, 300, [3, 5, 7])
    del out


def test_server_store_after_a_fill(fz):
    out = torch.zeros((ROWS, len(G)), dtype=torch.int32, device="cuda")
    with fz.Server(max_store_tuples=ROWS) as srv:
        t = srv.submit(dict(n=N, g=G, mode="store", out=out))
        r = srv.wait(t)
    assert r["status"] == 0 and r["written"] == ROWS
    assert all_elements(out, N, G)
    del out
