"""Python binding of libfz (include/fz.h): argument marshalling only.

Every step of the enumeration runs in the HIP kernels of ``libfz.so``; this
module converts Python integers, numpy arrays and torch tensors to the C ABI
and status codes to exceptions.  Importing it fails loudly when the library
has not been built (``python paper_2405_07989_amd/build.py``); there is no
fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfz.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "fz.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libfz.so not found at {LIB_PATH}: build it with `python paper_2405_07989_amd/build.py`")

# One HIP runtime per process: torch ships its own libamdhip64.so.7, and a
# second copy loaded from /opt/rocm would not see the device torch holds (nor
# share its pointers and streams).  Importing torch first makes the dynamic
# loader bind libfz.so's libamdhip64.so.7 to the copy already in memory.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

FZ_OK, FZ_TRUNCATED = 0, 1
FZ_EINVAL, FZ_EOVERFLOW, FZ_ENOMEM, FZ_EDEVICE, FZ_E2BIG, FZ_EINTERNAL = -1, -2, -3, -4, -5, -6
FZ_MAX_D = 16
FZ_MAX_LAST_GEN = 1 << 24


class FzError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        detail = ""
        if status in (FZ_EDEVICE, FZ_ENOMEM):
            detail = f" [{_lib.fz_last_error().decode()}]"
        super().__init__(f"{what}: {_lib.fz_strerror(status).decode()} (status {status}){detail}")


class fz_stats(ctypes.Structure):
    _fields_ = [("slices", ctypes.c_uint64), ("rows", ctypes.c_uint64),
                ("prefixes", ctypes.c_uint64), ("candidates", ctypes.c_uint64),
                ("elements", ctypes.c_uint64)]


class fz_slice_info(ctypes.Structure):
    _fields_ = [("elements", ctypes.c_uint64), ("rows", ctypes.c_uint64),
                ("prefixes", ctypes.c_uint64),
                ("t_begin", ctypes.c_uint64), ("t_end", ctypes.c_uint64),
                ("query", ctypes.c_uint32), ("slice", ctypes.c_uint32)]


class fz_query(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("g", ctypes.POINTER(ctypes.c_uint32)),
                ("d", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("target_len", ctypes.c_uint64), ("bins", ctypes.POINTER(ctypes.c_uint64)),
                ("nbins", ctypes.c_uint64), ("d_out", ctypes.c_void_p),
                ("max_tuples", ctypes.c_uint64)]


class fz_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("found", ctypes.c_int), ("count", ctypes.c_uint64),
                ("total", ctypes.c_uint64), ("min_len", ctypes.c_uint64),
                ("max_len", ctypes.c_uint64), ("written", ctypes.c_uint64)]


class fz_tune_result(ctypes.Structure):
    _fields_ = [("slices_per_wave", ctypes.c_uint32), ("workgroups_per_cu", ctypes.c_uint32),
                ("ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("candidates", ctypes.c_uint32)]


class fz_server_cfg(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("mem_budget", ctypes.c_uint64), ("max_store_tuples", ctypes.c_uint64)]


class fz_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("mean_batch", ctypes.c_double),
                ("p50_us", ctypes.c_double), ("p99_us", ctypes.c_double),
                ("max_us", ctypes.c_double), ("mean_us", ctypes.c_double),
                ("mean_phase1_us", ctypes.c_double), ("mean_phase2_us", ctypes.c_double)]


MODES = {"count": 0, "hist": 1, "exists": 2, "store": 3}

_u64, _u32, _i64 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_vp = ctypes.c_void_p

_SIGS = {
    "fz_count": (ctypes.c_int, [_u64, _u32p, _u32, _u64p]),
    "fz_count_stream": (ctypes.c_int, [_u64, _u32p, _u32, _u64p, _vp]),
    "fz_count_noalloc": (ctypes.c_int, [_u64, _u32p, _u32, _u64p, _vp]),
    "fz_length_bins": (ctypes.c_uint64, [_u64, _u32p, _u32]),
    "fz_length_hist": (ctypes.c_int, [_u64, _u32p, _u32, _u64p, _u64, _u64p, _u64p]),
    "fz_exists": (ctypes.c_int, [_u64, _u32p, _u32, _u64, ctypes.POINTER(ctypes.c_int)]),
    "fz_enumerate": (ctypes.c_int, [_u64, _u32p, _u32, _u32p, _u64, _u64p, _u64p]),
    "fz_enumerate_device": (ctypes.c_int, [_u64, _u32p, _u32, _vp, _u64, _u64p, _u64p, _vp]),
    "fz_unrank": (ctypes.c_int, [_u64, _u32p, _u32, _u64p, _u64, _u32p]),
    "fz_last_stats": (ctypes.c_int, [ctypes.POINTER(fz_stats)]),
    "fz_last_slices": (ctypes.c_int, [ctypes.POINTER(fz_slice_info), _u32,
                                      ctypes.POINTER(ctypes.c_uint32)]),
    "fz_config_set": (ctypes.c_int, [ctypes.c_char_p, _i64]),
    "fz_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "fz_profile_reset": (ctypes.c_int, []),
    "fz_profile_read": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), _u64p]),
    "fz_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "fz_batch": (ctypes.c_int, [ctypes.POINTER(fz_query), ctypes.POINTER(fz_result), _u32, _vp]),
    "fz_last_error": (ctypes.c_char_p, []),
    "fz_autotune": (ctypes.c_int, [ctypes.POINTER(fz_query), _u32, _u32,
                                   ctypes.POINTER(fz_tune_result)]),
    "fz_server_create": (ctypes.c_int, [ctypes.POINTER(fz_server_cfg),
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "fz_submit": (ctypes.c_int, [_vp, ctypes.POINTER(fz_query), _u64p]),
    "fz_wait": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(fz_result)]),
    "fz_server_stats_read": (ctypes.c_int, [_vp, ctypes.POINTER(fz_server_stats), ctypes.c_int]),
    "fz_server_destroy": (ctypes.c_int, [_vp]),
    "fz_probe_hbm_write": (ctypes.c_int, [ctypes.c_uint64, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]),
    "fz_probe_int_valu": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def exported_symbols_in_header() -> list[str]:
    """Names of the functions include/fz.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|uint64_t|const char \*)\s*(fz_\w+)\s*\(", text, re.M)))


def _gens(g):
    arr = np.ascontiguousarray(np.asarray(g, dtype=np.uint32).reshape(-1))
    return arr, arr.ctypes.data_as(_u32p)


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise FzError(rc, what)
    return rc


def _after_torch(stream):
    """The stream to queue library work on so that it runs after the caller's
    torch work (a fill of an output tensor, say): the given one; else torch's
    current stream; torch's default stream is the null stream, which the ABI
    cannot name (NULL selects the library's own, non-blocking stream), so its
    pending work is waited for instead."""
    if stream is not None or not torch.cuda.is_available():
        return stream
    cur = torch.cuda.current_stream()
    if cur.cuda_stream:
        return cur.cuda_stream
    cur.synchronize()
    return None


def count(n: int, g, stream=None) -> int:
    """|Z(n, g)| (fz_count / fz_count_stream)."""
    arr, gp = _gens(g)
    out = ctypes.c_uint64(0)
    if stream is None:
        _check(_lib.fz_count(n, gp, len(arr), ctypes.byref(out)), "fz_count")
    else:
        _check(_lib.fz_count_stream(n, gp, len(arr), ctypes.byref(out), _vp(stream)), "fz_count_stream")
    return out.value


def count_noalloc(n: int, g, stream=None) -> int:
    """|Z(n, g)| by fz_count_noalloc (no device allocation; the library's
    fixed scratch array).  stream: a hipStream_t handle, None for torch's
    current stream."""
    arr, gp = _gens(g)
    out = ctypes.c_uint64(0)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    _check(_lib.fz_count_noalloc(n, gp, len(arr), ctypes.byref(out), _vp(stream)),
           "fz_count_noalloc")
    return out.value


def length_bins(n: int, g) -> int:
    arr, gp = _gens(g)
    return int(_lib.fz_length_bins(n, gp, len(arr)))


def length_hist(n: int, g, nbins: int | None = None):
    """(bins, min_len, max_len); min/max are None when Z is empty."""
    arr, gp = _gens(g)
    nb = length_bins(n, g) if nbins is None else nbins
    bins = np.zeros(max(nb, 1), dtype=np.uint64)
    lo, hi = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(_lib.fz_length_hist(n, gp, len(arr), bins.ctypes.data_as(_u64p), nb,
                               ctypes.byref(lo), ctypes.byref(hi)), "fz_length_hist")
    if lo.value == 2**64 - 1:
        return bins[:nb], None, None
    return bins[:nb], lo.value, hi.value


def exists(n: int, g, target_len: int) -> bool:
    arr, gp = _gens(g)
    f = ctypes.c_int(0)
    _check(_lib.fz_exists(n, gp, len(arr), target_len, ctypes.byref(f)), "fz_exists")
    return bool(f.value)


def enumerate_host(n: int, g, max_tuples: int):
    """The min(|Z|, max_tuples) lex-smallest elements as a numpy array
    (fz_enumerate); returns (rows, total)."""
    arr, gp = _gens(g)
    d = len(arr)
    out = np.zeros((max(max_tuples, 1), d), dtype=np.uint32)
    total, written = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(_lib.fz_enumerate(n, gp, d, out.ctypes.data_as(_u32p), max_tuples,
                             ctypes.byref(total), ctypes.byref(written)), "fz_enumerate")
    return out[: written.value], total.value


def enumerate_device(n: int, g, out, max_tuples: int | None = None, stream=None):
    """Write the lex-smallest rows into ``out`` (a contiguous torch.int32 or
    uint32-compatible CUDA tensor of shape [rows, d]) on the current device
    (fz_enumerate_device), after the work already queued on torch's current
    stream (or on ``stream``).  Returns (total, written)."""
    arr, gp = _gens(g)
    d = len(arr)
    if out.dim() != 2 or out.shape[1] != d or not out.is_contiguous() or out.element_size() != 4:
        raise ValueError("out must be a contiguous [rows, d] tensor of 32-bit integers")
    cap = out.shape[0] if max_tuples is None else max_tuples
    if cap > out.shape[0]:
        raise ValueError("max_tuples exceeds the rows of out")
    total, written = ctypes.c_uint64(0), ctypes.c_uint64(0)
    stream = _after_torch(stream)
    _check(_lib.fz_enumerate_device(n, gp, d, _vp(out.data_ptr()), cap, ctypes.byref(total),
                                    ctypes.byref(written), _vp(stream) if stream else None),
           "fz_enumerate_device")
    return total.value, written.value


def unrank(n: int, g, ranks):
    """Element of each rank in ascending lex order (fz_unrank)."""
    arr, gp = _gens(g)
    r = np.ascontiguousarray(np.asarray(ranks, dtype=np.uint64).reshape(-1))
    out = np.zeros((max(len(r), 1), len(arr)), dtype=np.uint32)
    _check(_lib.fz_unrank(n, gp, len(arr), r.ctypes.data_as(_u64p), len(r), out.ctypes.data_as(_u32p)),
           "fz_unrank")
    return out[: len(r)]


def _struct_dtype(cls, kinds):
    """numpy dtype laid out exactly as the ctypes structure cls."""
    names = [f for f, _ in cls._fields_]
    return np.dtype({"names": names, "formats": [kinds[f] for f in names],
                     "offsets": [getattr(cls, f).offset for f in names],
                     "itemsize": ctypes.sizeof(cls)})


_QUERY_DT = _struct_dtype(fz_query, dict(n=np.uint64, g=np.uint64, d=np.uint32, mode=np.uint32,
                                         target_len=np.uint64, bins=np.uint64, nbins=np.uint64,
                                         d_out=np.uint64, max_tuples=np.uint64))
_RESULT_DT = _struct_dtype(fz_result, dict(status=np.int32, found=np.int32, count=np.uint64,
                                           total=np.uint64, min_len=np.uint64, max_len=np.uint64,
                                           written=np.uint64))


def _marshal(queries):
    """fz_query array for a list of query dicts (see batch); returns it with
    the host buffers it points to.  The array is filled column by column (a
    batch holds thousands of queries): all generators in one buffer, all
    histogram bins in another."""
    nq = len(queries)
    qa = np.zeros(max(nq, 1), dtype=_QUERY_DT)
    gl = [q["g"] for q in queries]
    ds = np.fromiter((len(g) for g in gl), dtype=np.int64, count=nq)
    allg = np.fromiter((x for g in gl for x in g), dtype=np.uint32, count=int(ds.sum()))
    goff = np.zeros(nq, dtype=np.uint64)
    if nq > 1:
        np.cumsum(ds[:-1], out=goff[1:], dtype=np.uint64)
    gbase = allg.ctypes.data if len(allg) else 0
    if nq:
        qa["n"][:nq] = [q["n"] for q in queries]
        qa["g"][:nq] = gbase + 4 * goff
        qa["d"][:nq] = ds
        qa["mode"][:nq] = [MODES[q["mode"]] for q in queries]
        qa["target_len"][:nq] = [q.get("target_len", 0) for q in queries]
    hist = [i for i, q in enumerate(queries) if q["mode"] == "hist"]
    nbs = []
    for i in hist:
        q = queries[i]
        nb = q.get("nbins")
        if not nb:
            g = q["g"]
            n = q["n"]
            # fz_length_bins' value, n // min g + 1, for a query plainly
            # inside the limits; the library decides every other one
            if 1 <= len(g) <= FZ_MAX_D and 0 <= n < 2**30 and min(g) >= 1 and \
                    n + 2 * max(max(g), n + 1 if len(g) == 1 else 0) < 2**31 and \
                    g[-1] <= FZ_MAX_LAST_GEN:
                nb = n // min(g) + 1
            else:
                gp = ctypes.cast(gbase + 4 * int(goff[i]), _u32p)
                nb = max(int(_lib.fz_length_bins(n, gp, int(ds[i]))), 1)
        nbs.append(nb)
    bins_all = np.zeros(sum(nbs), dtype=np.uint64)
    if hist:
        boff = np.zeros(len(hist), dtype=np.uint64)
        np.cumsum(np.asarray(nbs[:-1], dtype=np.uint64), out=boff[1:])
        qa["bins"][hist] = bins_all.ctypes.data + 8 * boff
        qa["nbins"][hist] = nbs
        for i, o, nb in zip(hist, boff.tolist(), nbs):
            queries[i]["_bins"] = bins_all[o:o + nb]
    for i, q in enumerate(queries):
        if q["mode"] != "store":
            continue
        out = q["out"]
        if out.dim() != 2 or out.shape[1] != int(ds[i]) or not out.is_contiguous() \
                or out.element_size() != 4:
            raise ValueError("out must be a contiguous [rows, d] tensor of 32-bit integers")
        mt = q.get("max_tuples", out.shape[0])
        if mt > out.shape[0]:
            raise ValueError("max_tuples exceeds the rows of out")
        qa["d_out"][i] = out.data_ptr()
        qa["max_tuples"][i] = mt
    qarr = (fz_query * max(nq, 1)).from_buffer(qa)
    return qarr, [qa, allg, bins_all]


def batch(queries, stream=None):
    """Run a list of queries as one batch (fz_batch).  Each query is a dict:
    n, g, mode ('count' | 'hist' | 'exists' | 'store'), target_len (exists),
    out (store: a contiguous [rows, d] 32-bit CUDA tensor), max_tuples (store,
    default: out's rows).  Returns one dict per query: status, count, total,
    found, and bins / min_len / max_len (hist) or written (store).  The batch
    runs after the work already queued on torch's current stream (or on
    ``stream``)."""
    nq = len(queries)
    qarr, keep = _marshal(queries)
    rarr = (fz_result * max(nq, 1))()
    if nq:
        stream = _after_torch(stream)
    _check(_lib.fz_batch(qarr, rarr, nq, _vp(stream) if stream else None), "fz_batch")
    res = np.frombuffer(rarr, dtype=_RESULT_DT, count=nq)
    return [_result_dict(q, r) for q, r in zip(queries, res.tolist())]


def autotune(queries, reps: int = 3) -> dict:
    """fz_autotune: time the queries (one batch, or the single-query path for
    one query) under each candidate (slices per wave, workgroups per CU) and
    keep the fastest for this process.  Returns the chosen pair and times."""
    qarr, keep = _marshal(queries)
    out = fz_tune_result()
    _check(_lib.fz_autotune(qarr, len(queries), reps, ctypes.byref(out)), "fz_autotune")
    for q in queries:
        q.pop("_bins", None)
    return {k: getattr(out, k) for k, _ in fz_tune_result._fields_}


def _result_dict(q, r):
    """Result dict of one query from its fz_result, as a ctypes structure or
    as a tuple in field order (status, found, count, total, min_len,
    max_len, written)."""
    if not isinstance(r, tuple):
        r = tuple(getattr(r, f) for f, _ in fz_result._fields_)
    status, found, count, total, min_len, max_len, written = r
    d = dict(status=status, count=count, total=total, found=bool(found))
    if q["mode"] == "hist":
        d["bins"] = q.pop("_bins", None)
        d["min_len"] = None if min_len == 2**64 - 1 else min_len
        d["max_len"] = None if min_len == 2**64 - 1 else max_len
    if q["mode"] == "store":
        d["written"] = written
    return d


class Server:
    """fz_server: submit queries (dicts as for batch) one at a time, collect
    each result with wait(ticket).  The library's own thread batches what has
    arrived onto up to max_inflight streams."""

    def __init__(self, max_inflight=0, max_batch=0, mem_budget=0, max_store_tuples=0):
        cfg = fz_server_cfg(max_inflight, max_batch, mem_budget, max_store_tuples)
        h = ctypes.c_void_p()
        _check(_lib.fz_server_create(ctypes.byref(cfg), ctypes.byref(h)), "fz_server_create")
        self._h = h
        self._live = {}  # ticket -> (query, host buffers it points to)

    def submit(self, q, sync: bool = True) -> int:
        """Queue one query; returns its ticket.  The server runs on streams of
        its own, so a store query's output must be ready when it is
        submitted: with sync (the default) this waits for torch's current
        stream first; pass sync=False when the outputs are known to be ready
        (allocated without a kernel, or synchronized once beforehand)."""
        if sync and q.get("out") is not None and torch.cuda.is_available():
            torch.cuda.current_stream().synchronize()
        qarr, keep = _marshal([q])
        t = ctypes.c_uint64(0)
        _check(_lib.fz_submit(self._h, qarr, ctypes.byref(t)), "fz_submit")
        self._live[t.value] = (q, keep)
        return t.value

    def wait(self, ticket: int) -> dict:
        r = fz_result()
        _check(_lib.fz_wait(self._h, ticket, ctypes.byref(r)), "fz_wait")
        q, _ = self._live.pop(ticket)
        return _result_dict(q, r)

    def stats(self, reset=False) -> dict:
        st = fz_server_stats()
        _check(_lib.fz_server_stats_read(self._h, ctypes.byref(st), 1 if reset else 0),
               "fz_server_stats_read")
        return {k: getattr(st, k) for k, _ in fz_server_stats._fields_}

    def close(self):
        if self._h:
            _check(_lib.fz_server_destroy(self._h), "fz_server_destroy")
            self._h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def last_stats() -> dict:
    s = fz_stats()
    _check(_lib.fz_last_stats(ctypes.byref(s)), "fz_last_stats")
    return {k: getattr(s, k) for k, _ in fz_stats._fields_}


def last_slices():
    """Per-slice records of the last enumeration as a numpy structured array
    (elements, rows, prefixes, t_begin, t_end, query, slice; clocks in 100 MHz
    ticks)."""
    n = ctypes.c_uint32(0)
    _check(_lib.fz_last_slices(None, 0, ctypes.byref(n)), "fz_last_slices")
    buf = (fz_slice_info * max(n.value, 1))()
    _check(_lib.fz_last_slices(buf, n.value, ctypes.byref(n)), "fz_last_slices")
    arr = np.ctypeslib.as_array(buf)[: n.value]
    return arr.copy()


def config_set(key: str, value: int) -> None:
    _check(_lib.fz_config_set(key.encode(), value), f"fz_config_set({key})")


def profile_enable(on: bool = True) -> None:
    _check(_lib.fz_profile_enable(1 if on else 0), "fz_profile_enable")


def profile_reset() -> None:
    _check(_lib.fz_profile_reset(), "fz_profile_reset")


def profile_read(kernel: str):
    """(total_ms, launches) of one kernel since the last reset."""
    ms, n = ctypes.c_double(0), ctypes.c_uint64(0)
    _check(_lib.fz_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)), "fz_profile_read")
    return ms.value, n.value


def probe_int_valu() -> dict:
    """fz_probe_int_valu: the device's sustained int32 vector-ALU rate."""
    rate, ms = ctypes.c_double(0), ctypes.c_double(0)
    _check(_lib.fz_probe_int_valu(ctypes.byref(rate), ctypes.byref(ms)), "fz_probe_int_valu")
    return {"lane_ops_per_s": rate.value, "ms": ms.value}


def probe_hbm_write(nbytes: int = 12 * 10**9) -> dict:
    """fz_probe_hbm_write: the device's sustained HBM write rate."""
    rate, ms = ctypes.c_double(0), ctypes.c_double(0)
    _check(_lib.fz_probe_hbm_write(nbytes, ctypes.byref(rate), ctypes.byref(ms)),
           "fz_probe_hbm_write")
    return {"bytes_per_s": rate.value, "ms": ms.value}


def strerror(status: int) -> str:
    return _lib.fz_strerror(status).decode()
