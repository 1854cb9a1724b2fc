"""The C ABI on the CPU: libfz.so loads, exports every function include/fz.h
declares, and rejects invalid input before touching a device."""
import ctypes
import subprocess

import numpy as np
import pytest

import paper_2405_07989_amd as fz


def test_header_declares_the_entry_points():
    names = fz.exported_symbols_in_header()
    for want in ["fz_count", "fz_length_hist", "fz_exists", "fz_enumerate", "fz_enumerate_device",
                 "fz_unrank", "fz_strerror", "fz_length_bins"]:
        assert want in names


def test_every_declared_symbol_is_exported():
    out = subprocess.run(["nm", "-D", "--defined-only", fz.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in fz.exported_symbols_in_header():
        assert name in exported, name
        assert hasattr(fz._lib, name)


def _g(g):
    a = np.asarray(g, dtype=np.uint32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def test_validation_errors_without_a_device():
    L = fz._lib
    c = ctypes.c_uint64(123)
    a, gp = _g([3, 5])
    assert L.fz_count(10, None, 2, ctypes.byref(c)) == fz.FZ_EINVAL
    assert L.fz_count(10, gp, 0, ctypes.byref(c)) == fz.FZ_EINVAL
    assert L.fz_count(10, gp, 2, None) == fz.FZ_EINVAL
    z, zp = _g([3, 0, 5])
    assert L.fz_count(10, zp, 3, ctypes.byref(c)) == fz.FZ_EINVAL
    big, bp = _g(list(range(1, 18)))
    assert L.fz_count(10, bp, 17, ctypes.byref(c)) == fz.FZ_EINVAL  # d > FZ_MAX_D
    assert L.fz_count(2**31 - 3, gp, 2, ctypes.byref(c)) == fz.FZ_EOVERFLOW
    assert L.fz_count(2**30, gp, 2, ctypes.byref(c)) == fz.FZ_EOVERFLOW  # d <= 2 limit
    h, hp = _g([3, 2**24 + 1])
    assert L.fz_count(10, hp, 2, ctypes.byref(c)) == fz.FZ_E2BIG
    assert c.value == 123  # untouched on error
    bins = np.zeros(3, dtype=np.uint64)
    lo, hi = ctypes.c_uint64(0), ctypes.c_uint64(0)
    a3, g3 = _g([3, 5, 7])
    assert fz._lib.fz_length_bins(100, g3, 3) == 100 // 3 + 1
    assert L.fz_length_hist(100, g3, 3, bins.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), 3,
                            ctypes.byref(lo), ctypes.byref(hi)) == fz.FZ_EINVAL
    assert L.fz_exists(100, g3, 3, 5, None) == fz.FZ_EINVAL
    assert L.fz_enumerate(100, g3, 3, None, 5, ctypes.byref(c), ctypes.byref(c)) == fz.FZ_EINVAL
    r = np.array([0], dtype=np.uint64)
    assert L.fz_unrank(100, g3, 3, None, 1, None) == fz.FZ_EINVAL
    assert L.fz_config_set(b"no_such_knob", 1) == fz.FZ_EINVAL
    assert L.fz_config_set(b"slices_per_wave", -1) == fz.FZ_EINVAL
    assert fz._lib.fz_length_bins(10, None, 2) == 0


def test_limit_check_does_not_wrap():
    """n near 2^64 must be refused: n + 2 max g wraps in 64 bits, so each
    term is bounded on its own before the sum."""
    L = fz._lib
    c = ctypes.c_uint64(7)
    for n, g in [(2**64 - 2, [1, 1, 1]), (2**64 - 1500, [1000, 999, 998, 997]),
                 (2**64 - 1, [5]), (2**63, [3, 5]), (2**32, [3, 5, 7]), (2**31, [3, 5, 7])]:
        a, gp = _g(g)
        assert L.fz_length_bins(n, gp, len(g)) == 0, n
        assert L.fz_count(n, gp, len(g), ctypes.byref(c)) == fz.FZ_EOVERFLOW, n
        assert L.fz_exists(n, gp, len(g), 1, ctypes.byref(ctypes.c_int(0))) == fz.FZ_EOVERFLOW
        assert c.value == 7
    # the largest accepted n still passes validation (the device call itself
    # is what fails without a GPU)
    a, gp = _g([3, 5, 7])
    assert L.fz_length_bins(2**31 - 15, gp, 3) == (2**31 - 15) // 3 + 1
    assert L.fz_length_bins(2**31 - 14, gp, 3) == 0


def test_strerror_covers_every_status():
    for s in [0, 1, -1, -2, -3, -4, -5, -6]:
        assert fz.strerror(s) and fz.strerror(s) != "unknown status"
    assert fz.strerror(99) == "unknown status"


def test_no_device_is_a_clean_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(fz.FzError) as e:
        fz.count(100, [3, 5, 7])
    assert e.value.status == fz.FZ_EDEVICE


def test_probe_validation():
    L = fz._lib
    assert L.fz_probe_int_valu(None, None) == fz.FZ_EINVAL
    import torch
    if not torch.cuda.is_available():
        rate = ctypes.c_double(0)
        assert L.fz_probe_int_valu(ctypes.byref(rate), None) == fz.FZ_EDEVICE


def test_batch_validation_without_a_device():
    L = fz._lib
    assert L.fz_batch(None, None, 0, None) == fz.FZ_OK
    r = (fz.fz_result * 1)()
    q = (fz.fz_query * 1)()
    assert L.fz_batch(None, r, 1, None) == fz.FZ_EINVAL
    assert L.fz_batch(q, None, 1, None) == fz.FZ_EINVAL
    assert fz.batch([]) == []
    import torch
    if not torch.cuda.is_available():
        with pytest.raises(fz.FzError) as e:
            fz.batch([dict(n=10, g=[3, 5], mode="count")])
        assert e.value.status == fz.FZ_EDEVICE


def test_server_validation_without_a_device():
    L = fz._lib
    assert L.fz_server_create(None, None) == fz.FZ_EINVAL
    cfg = fz.fz_server_cfg(9, 0, 0, 0)  # more than 8 launch slots
    h = ctypes.c_void_p()
    assert L.fz_server_create(ctypes.byref(cfg), ctypes.byref(h)) == fz.FZ_EINVAL
    assert L.fz_submit(None, None, None) == fz.FZ_EINVAL
    assert L.fz_wait(None, 1, None) == fz.FZ_EINVAL
    assert L.fz_server_destroy(None) == fz.FZ_EINVAL
    import torch
    if not torch.cuda.is_available():
        with pytest.raises(fz.FzError) as e:
            fz.Server()
        assert e.value.status == fz.FZ_EDEVICE
