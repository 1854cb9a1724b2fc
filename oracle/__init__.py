"""CPU oracle for the factorization set Z(n, (g_1..g_d)) (paper Sec. 1).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package; the GPU library
never does, and the two share no code.  The arithmetic lives in plain C
(``fz_oracle.c``); this module only marshals arguments.

Functions:
  walk / count / hist / exists / store / store_from   ascending-lex nested loops
  dp_count, dp_hist     generating-function coefficients (exact, u64)
  unrank_dp             r-th element of Z in ascending lex order
  candidate_stream      the paper's descending candidate stream (Alg. 3.1),
                        optionally with the modulo skip (Sec. 3.2.4)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fz_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, EOVERFLOW, ENOMEM, EINTERNAL = 0, -1, -2, -3, -4


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile fz_oracle.c into liboracle.so with gcc (plain -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


class library:
    """Context manager that points this module at another build of the oracle
    source (used by the tests that plant mistakes in a copy of it)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _L():
    global _lib
    if _lib is None:
        build()
        _lib = _load(_LIB)
    return _lib


def _load(path):
    lib = ctypes.CDLL(path)
    u64, u32p, u64p, ip = (ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32),
                           ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int))
    lib.fzo_walk.argtypes = [u64, u32p, ctypes.c_uint32, u32p, u64, u64p, u64p, u64, ip,
                             u64, ip, u32p, u64, u64p]
    lib.fzo_dp_count.argtypes = [u64, u32p, ctypes.c_uint32, u64p]
    lib.fzo_dp_hist.argtypes = [u64, u32p, ctypes.c_uint32, u64p, u64]
    lib.fzo_dp_series.argtypes = [u64, u32p, ctypes.c_uint32, u64p]
    lib.fzo_unrank_dp.argtypes = [u64, u32p, ctypes.c_uint32, u64, u32p]
    lib.fzo_candidate_stream.argtypes = [u64, u32p, ctypes.c_uint32, u32p, u32p, ctypes.c_int,
                                         u32p, u64, u64p, u64p, u64p]
    for f in (lib.fzo_walk, lib.fzo_dp_count, lib.fzo_dp_hist, lib.fzo_dp_series,
              lib.fzo_unrank_dp, lib.fzo_candidate_stream):
        f.restype = ctypes.c_int
    return lib


def _g(g):
    arr = np.ascontiguousarray(np.asarray(g, dtype=np.uint32))
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _check(rc, what):
    if rc == EOVERFLOW:
        raise OverflowError(f"{what}: count does not fit in 64 bits")
    if rc != OK:
        raise OracleError(f"{what}: oracle status {rc}")


def max_len(n: int, g) -> int:
    """Largest possible length sum(a_i) of an element of Z(n, g)."""
    return n // min(g)


def walk(n, g, *, start=None, stop_after=0, nbins=0, target_len=None, out_cap=0):
    """Ascending-lex walk over Z(n,g) (optionally from ``start``, stopping after
    ``stop_after`` elements).  Returns dict(count, hist, hist_oor, found, store)."""
    L = _L()
    garr, gp = _g(g)
    d = len(garr)
    cnt = ctypes.c_uint64(0)
    written = ctypes.c_uint64(0)
    found = ctypes.c_int(0)
    oor = ctypes.c_int(0)
    hist = np.zeros(max(nbins, 1), dtype=np.uint64)
    out = np.zeros((max(out_cap, 1), d), dtype=np.uint32)
    if start is not None:
        sarr, sp = _g(start)
    else:
        sarr, sp = None, None
    tl = np.uint64(2**64 - 1) if target_len is None else np.uint64(target_len)
    rc = L.fzo_walk(n, gp, d, sp, stop_after, ctypes.byref(cnt),
                    hist.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)) if nbins else None,
                    nbins, ctypes.byref(oor), int(tl), ctypes.byref(found),
                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)) if out_cap else None,
                    out_cap, ctypes.byref(written))
    _check(rc, "walk")
    return dict(count=cnt.value, hist=hist[:nbins] if nbins else None, hist_oor=bool(oor.value),
                found=bool(found.value), store=out[: written.value] if out_cap else None)


def count(n, g) -> int:
    return walk(n, g)["count"]


def hist(n, g, nbins=None):
    """Length histogram by enumeration: (bins, min_len, max_len); empty Z gives
    (zeros, None, None)."""
    nb = max_len(n, g) + 1 if nbins is None else nbins
    h = walk(n, g, nbins=nb)["hist"]
    nz = np.nonzero(h)[0]
    if len(nz) == 0:
        return h, None, None
    return h, int(nz[0]), int(nz[-1])


def exists(n, g, target_len) -> bool:
    return walk(n, g, target_len=target_len)["found"]


def store(n, g, max_tuples=None):
    """The first ``max_tuples`` elements (all if None) in ascending lex order."""
    cap = count(n, g) if max_tuples is None else max_tuples
    return walk(n, g, out_cap=cap, stop_after=cap)["store"] if cap else np.zeros((0, len(g)), np.uint32)


def store_from(n, g, start, k):
    """The k lex-smallest elements that are >=_lex start."""
    if k == 0:
        return np.zeros((0, len(g)), np.uint32)
    return walk(n, g, start=start, out_cap=k, stop_after=k)["store"]


def dp_count(n, g) -> int:
    L = _L()
    garr, gp = _g(g)
    c = ctypes.c_uint64(0)
    _check(L.fzo_dp_count(n, gp, len(garr), ctypes.byref(c)), "dp_count")
    return c.value


def dp_series(nmax, g):
    """|Z(v, g)| for v = 0..nmax (2**64-1 marks overflow)."""
    L = _L()
    garr, gp = _g(g)
    s = np.zeros(nmax + 1, dtype=np.uint64)
    _check(L.fzo_dp_series(nmax, gp, len(garr), s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))),
           "dp_series")
    return s


def dp_hist(n, g, nbins=None):
    L = _L()
    garr, gp = _g(g)
    nb = max_len(n, g) + 1 if nbins is None else nbins
    h = np.zeros(nb, dtype=np.uint64)
    _check(L.fzo_dp_hist(n, gp, len(garr), h.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), nb),
           "dp_hist")
    return h


def unrank_dp(n, g, r):
    L = _L()
    garr, gp = _g(g)
    out = np.zeros(len(garr), dtype=np.uint32)
    _check(L.fzo_unrank_dp(n, gp, len(garr), r, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))),
           "unrank_dp")
    return out


def candidate_stream(n, g, *, start=None, bound=None, use_modulo=False, cap=None):
    """Run the paper's candidate stream.  Returns dict(valid (descending rows),
    n_valid, n_cand, max_coord)."""
    L = _L()
    garr, gp = _g(g)
    d = len(garr)
    if cap is None:
        cap = dp_count(n, g)
    valid = np.zeros((max(cap, 1), d), dtype=np.uint32)
    nv = ctypes.c_uint64(0)
    nc = ctypes.c_uint64(0)
    mc = np.zeros(d, dtype=np.uint64)
    sarr, sp = _g(start) if start is not None else (None, None)
    barr, bp = _g(bound) if bound is not None else (None, None)
    rc = L.fzo_candidate_stream(n, gp, d, sp, bp, 1 if use_modulo else 0,
                                valid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), cap,
                                ctypes.byref(nv), ctypes.byref(nc),
                                mc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    _check(rc, "candidate_stream")
    return dict(valid=valid[: min(nv.value, cap)], n_valid=nv.value, n_cand=nc.value, max_coord=mc)
