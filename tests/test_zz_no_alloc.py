"""The allocation-free count (fz_count_noalloc) against fz_count_stream, the
entry point it is a variant of: the same results on calls in a row (the
second smaller, so it reads the fixed array after a larger call left it
full), and a clear refusal of a query beyond the array's size."""
import ctypes

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fz():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the gpu tests need an MI355X")
    import paper_2405_07989_amd as m
    return m


def _noalloc(fz, n, g, stream):
    arr = np.ascontiguousarray(np.asarray(g, dtype=np.uint32))
    out = ctypes.c_uint64(0)
    rc = fz._lib.fz_count_noalloc(n, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                  len(arr), ctypes.byref(out), ctypes.c_void_p(stream))
    return rc, out.value


@pytest.mark.parametrize("seq", [
    # (n, g) pairs called in a row, each later one smaller than the one before
    [(100000, [108, 86, 164, 185, 145, 65]), (10000, [11, 13, 17, 23])],
    [(10000, [11, 13, 17, 23]), (300, [3, 5, 7])],
    [(20000, [13, 37, 38, 40, 41, 42, 43, 44]), (77, [2, 9, 11, 4]), (0, [5, 7])],
    [(5000, [7]), (4999, [7])],
])
def test_noalloc_matches_count_stream(fz, seq):
    s = torch.cuda.Stream()
    for n, g in seq:
        want = fz.count(n, g, stream=s.cuda_stream)
        rc, got = _noalloc(fz, n, g, s.cuda_stream)
        assert rc == 0 and got == want, (n, g, rc, got, want)
        # and on the null stream
        rc, got = _noalloc(fz, n, g, 0)
        assert rc == 0 and got == want, (n, g)
    if seq[-1][0] <= 10000:
        n, g = seq[-1]
        assert got == oracle.dp_count(n, g)


def test_noalloc_binding_and_sparse_and_pair_sets(fz):
    # row skipping and the pair table use the count table from the array too
    from test_gpu_parity import SPARSE
    for n, g in SPARSE[:4]:
        assert fz.count_noalloc(n, g) == fz.count(n, g) == oracle.dp_count(n, g)


def test_noalloc_refuses_beyond_the_array(fz):
    # tables of (2d - 3)(n + 1) 8 bytes = 3 x 8e6 x 8 = 192 MB > 64 MB
    rc, got = _noalloc(fz, 8_000_000, [3, 5, 7], 0)
    assert rc == fz.FZ_E2BIG and got == 0
    assert "FZ_NOALLOC_SCRATCH_BYTES" in fz._lib.fz_last_error().decode()
    # the array still works afterwards
    rc, got = _noalloc(fz, 10000, [11, 13, 17, 23], 0)
    assert rc == 0 and got == 3009519
    # invalid input is refused before any device work, as fz_count
    rc, _ = _noalloc(fz, 10, [3, 0], 0)
    assert rc == fz.FZ_EINVAL
