"""Thin ctypes binding of libswalign.so (include/swalign.h).

Argument marshalling only: every step of the alignment runs in the HIP
library.  PyTorch provides device memory and streams.  The functions keep the
C names (sw_create, sw_align_batch, ...); ``Aligner`` wraps them for torch
tensors.  There is no CPU fallback: if the library is missing or no GPU is
present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswalign.so")

SW_OK = 0
SW_PENDING = 1
SW_EINVAL = -1
SW_ENOMEM = -2
SW_ETOOLONG = -3
SW_EDEVICE = -4
SW_EINTERNAL = -5
SW_MAX_QUERY = 2048
SW_MAX_REF = 60000
SW_MAX_ALPHABET = 31
SW_MAX_SCHEMES = 4
SW_NOALLOC_MAX_PAIRS = 1 << 20

_ERRNAMES = {SW_EINVAL: "SW_EINVAL", SW_ENOMEM: "SW_ENOMEM", SW_ETOOLONG: "SW_ETOOLONG",
             SW_EDEVICE: "SW_EDEVICE", SW_EINTERNAL: "SW_EINTERNAL"}

EXPORTED = ("sw_create", "sw_destroy", "sw_last_error", "sw_set_option", "sw_get_option",
            "sw_align_batch", "sw_align_batch_noalloc", "sw_submit", "sw_poll", "sw_align_spans", "sw_last_stats", "sw_last_timing", "sw_last_host_timing", "sw_last_bin_stats",
            "sw_shapes", "sw_set_routing", "sw_get_routing", "sw_align_cigar", "sw_last_cigar_stats", "sw_search",
            "sw_server_create", "sw_server_destroy", "sw_server_last_error", "sw_server_submit",
            "sw_server_poll", "sw_server_stats", "sw_server_timing")


class sw_result(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int32), ("q_start", ctypes.c_int32), ("q_end", ctypes.c_int32),
                ("r_start", ctypes.c_int32), ("r_end", ctypes.c_int32)]


class sw_scheme(ctypes.Structure):
    _fields_ = [("matrix", ctypes.c_void_p), ("alphabet", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32)]


class sw_batch(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_void_p), ("q_off", ctypes.c_void_p), ("refs", ctypes.c_void_p),
                ("r_off", ctypes.c_void_p), ("scheme_id", ctypes.c_void_p), ("n_pairs", ctypes.c_int64)]


class sw_bin_stat(ctypes.Structure):
    _fields_ = [("pass_", ctypes.c_int32), ("precision", ctypes.c_int32), ("lanes", ctypes.c_int32),
                ("rows", ctypes.c_int32), ("pairs", ctypes.c_int64), ("cells", ctypes.c_int64),
                ("ms", ctypes.c_float), ("column", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("launch", ctypes.c_int32), ("family_hi", ctypes.c_int32), ("family_lo", ctypes.c_int32),
                ("family_waves", ctypes.c_int32)]


class SwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_ERRNAMES.get(code, str(code)), msg))
        self.code = code


_lib = None


def _init_torch_runtime():
    """PyTorch carries its own copy of the HIP runtime beside the system one
    the library links.  Both work in one process when PyTorch's is
    initialised first (the other order leaves PyTorch without devices), so
    it is initialised before the library is loaded; without a GPU this is a
    no-op."""
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except Exception:   # noqa: BLE001 -- no GPU or no torch: nothing to order
        pass


def load_library(path: str = LIB_PATH):
    """Load libswalign.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libswalign.so is not built (run __graft_entry__.build() or "
                           "python paper_2208_12350_amd/build.py)")
    _init_torch_runtime()
    lib = ctypes.CDLL(path)
    lib.sw_create.restype = ctypes.c_void_p
    lib.sw_create.argtypes = [ctypes.c_int, ctypes.c_char_p]
    lib.sw_destroy.restype = None
    lib.sw_destroy.argtypes = [ctypes.c_void_p]
    lib.sw_last_error.restype = ctypes.c_char_p
    lib.sw_last_error.argtypes = [ctypes.c_void_p]
    lib.sw_set_option.restype = ctypes.c_int
    lib.sw_set_option.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int64]
    lib.sw_get_option.restype = ctypes.c_int
    lib.sw_get_option.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)]
    lib.sw_align_batch.restype = ctypes.c_int
    lib.sw_align_batch.argtypes = [ctypes.c_void_p, ctypes.POINTER(sw_batch), ctypes.POINTER(sw_scheme),
                                   ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.sw_align_batch_noalloc.restype = ctypes.c_int
    lib.sw_align_batch_noalloc.argtypes = [ctypes.c_void_p, ctypes.POINTER(sw_batch), ctypes.POINTER(sw_scheme),
                                           ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.sw_submit.restype = ctypes.c_int
    lib.sw_submit.argtypes = [ctypes.c_void_p, ctypes.POINTER(sw_batch), ctypes.POINTER(sw_scheme), ctypes.c_int,
                              ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]
    lib.sw_poll.restype = ctypes.c_int
    lib.sw_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int]
    lib.sw_align_spans.restype = ctypes.c_int
    lib.sw_align_spans.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 7 + [ctypes.c_int64, ctypes.POINTER(sw_scheme),
                                                                             ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.sw_last_stats.restype = ctypes.c_int
    lib.sw_last_stats.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 3
    lib.sw_last_timing.restype = ctypes.c_int
    lib.sw_last_timing.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_float)] * 3
    I32P = ctypes.POINTER(ctypes.c_int32)
    lib.sw_last_host_timing.restype = ctypes.c_int
    lib.sw_last_host_timing.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_double)] * 2
    lib.sw_shapes.restype = ctypes.c_int
    lib.sw_shapes.argtypes = [ctypes.c_void_p, I32P, I32P, I32P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.sw_set_routing.restype = ctypes.c_int
    lib.sw_set_routing.argtypes = [ctypes.c_void_p, ctypes.c_int, I32P, I32P, I32P, ctypes.c_int]
    lib.sw_get_routing.restype = ctypes.c_int
    lib.sw_get_routing.argtypes = [ctypes.c_void_p, ctypes.c_int, I32P, I32P, I32P, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_int)]
    lib.sw_last_bin_stats.restype = ctypes.c_int
    lib.sw_last_bin_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(sw_bin_stat), ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int)]
    lib.sw_align_cigar.restype = ctypes.c_int
    lib.sw_align_cigar.argtypes = [ctypes.c_void_p, ctypes.POINTER(sw_batch), ctypes.POINTER(sw_scheme),
                                   ctypes.c_int] + [ctypes.c_void_p] * 5
    lib.sw_last_cigar_stats.restype = ctypes.c_int
    lib.sw_last_cigar_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]
    lib.sw_search.restype = ctypes.c_int
    lib.sw_search.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_int64, ctypes.POINTER(sw_scheme), ctypes.c_void_p, ctypes.c_void_p]
    lib.sw_server_create.restype = ctypes.c_void_p
    lib.sw_server_create.argtypes = [ctypes.c_int, ctypes.POINTER(sw_scheme), ctypes.c_int, ctypes.c_int64,
                                     ctypes.c_int, ctypes.c_int64, ctypes.c_char_p]
    lib.sw_server_timing.restype = ctypes.c_int
    lib.sw_server_timing.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_double)] * 3
    lib.sw_server_destroy.restype = None
    lib.sw_server_destroy.argtypes = [ctypes.c_void_p]
    lib.sw_server_last_error.restype = ctypes.c_char_p
    lib.sw_server_last_error.argtypes = [ctypes.c_void_p]
    lib.sw_server_submit.restype = ctypes.c_int
    lib.sw_server_submit.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 5 + [ctypes.c_int64,
                                                                                ctypes.POINTER(ctypes.c_uint64)]
    lib.sw_server_poll.restype = ctypes.c_int
    lib.sw_server_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_double)]
    lib.sw_server_stats.restype = ctypes.c_int
    lib.sw_server_stats.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 5
    _lib = lib
    return lib


# ---- C-named wrappers --------------------------------------------------------

def sw_create(device: int = 0, tuning: Optional[str] = None) -> int:
    h = load_library().sw_create(device, tuning.encode() if tuning else None)
    if not h:
        raise RuntimeError("sw_create(%d) failed (no such HIP device or bad tuning string)" % device)
    return h


def sw_destroy(h: int) -> None:
    load_library().sw_destroy(h)


def sw_last_error(h: int) -> str:
    return load_library().sw_last_error(h).decode(errors="replace")


def _check(h, rc):
    if rc != SW_OK:
        raise SwError(rc, sw_last_error(h))
    return rc


def sw_set_option(h: int, key: str, value: int) -> None:
    _check(h, load_library().sw_set_option(h, key.encode(), int(value)))


def sw_get_option(h: int, key: str) -> int:
    v = ctypes.c_int64(0)
    _check(h, load_library().sw_get_option(h, key.encode(), ctypes.byref(v)))
    return int(v.value)


def sw_align_batch(h: int, batch: sw_batch, schemes, n_schemes: int, out_ptr: int, stream_ptr) -> int:
    """Raw call; returns the status code (does not raise)."""
    return load_library().sw_align_batch(h, ctypes.byref(batch), schemes, n_schemes, out_ptr, stream_ptr)


def sw_align_batch_noalloc(h: int, batch: sw_batch, schemes, n_schemes: int, out_ptr: int, stream_ptr) -> int:
    """Raw call of the allocation-free variant; returns the status code."""
    return load_library().sw_align_batch_noalloc(h, ctypes.byref(batch), schemes, n_schemes, out_ptr, stream_ptr)


def sw_submit(h: int, batch: sw_batch, schemes, n_schemes: int, out_ptr, stream_ptr):
    """Raw call; returns (status, ticket)."""
    t = ctypes.c_uint64(0)
    rc = load_library().sw_submit(h, ctypes.byref(batch), schemes, n_schemes, out_ptr, stream_ptr, ctypes.byref(t))
    return rc, int(t.value)


def sw_poll(h: int, ticket: int, wait: int) -> int:
    """Raw call; returns the status code (SW_PENDING while the call runs)."""
    return load_library().sw_poll(h, ticket, wait)


def sw_align_spans(h: int, queries, q_beg, q_end, refs, r_beg, r_end, scheme_id, n_pairs: int, schemes,
                   n_schemes: int, out_ptr, stream_ptr) -> int:
    """Raw call with device pointers; returns the status code."""
    return load_library().sw_align_spans(h, queries, q_beg, q_end, refs, r_beg, r_end, scheme_id, n_pairs,
                                         schemes, n_schemes, out_ptr, stream_ptr)


def sw_align_cigar(h: int, batch: sw_batch, schemes, n_schemes: int, out_ptr, cigar_off_ptr, cigar_ptr,
                   cigar_len_ptr, stream_ptr) -> int:
    """Raw call with device pointers; returns the status code."""
    return load_library().sw_align_cigar(h, ctypes.byref(batch), schemes, n_schemes, out_ptr, cigar_off_ptr,
                                         cigar_ptr, cigar_len_ptr, stream_ptr)


def sw_last_cigar_stats(h: int):
    """(box_cells, record_bytes, chunks, sweep_ms, walk_ms) of the last
    sw_align_cigar call."""
    c, b, k = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int32(0)
    s, w = ctypes.c_float(0), ctypes.c_float(0)
    _check(h, load_library().sw_last_cigar_stats(h, ctypes.byref(c), ctypes.byref(b), ctypes.byref(k),
                                                 ctypes.byref(s), ctypes.byref(w)))
    return int(c.value), int(b.value), int(k.value), float(s.value), float(w.value)


def sw_last_stats(h: int):
    f, r, i = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _check(h, load_library().sw_last_stats(h, ctypes.byref(f), ctypes.byref(r), ctypes.byref(i)))
    return int(f.value), int(r.value), int(i.value)


def sw_last_timing(h: int):
    a, b, c = ctypes.c_float(0), ctypes.c_float(0), ctypes.c_float(0)
    _check(h, load_library().sw_last_timing(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return float(a.value), float(b.value), float(c.value)


def sw_last_bin_stats(h: int):
    """Per-bin statistics of the last call: a list of dicts with keys
    pass, precision, lanes, rows, column, tile, pairs, cells, ms, launch,
    family_hi, family_lo, family_waves (bins one family launch swept share
    launch and ms)."""
    lib = load_library()
    n = ctypes.c_int(0)
    lib.sw_last_bin_stats(h, None, 0, ctypes.byref(n))
    arr = (sw_bin_stat * max(1, n.value))()
    _check(h, lib.sw_last_bin_stats(h, arr, n.value, ctypes.byref(n)))
    return [{"pass": e.pass_, "precision": e.precision, "lanes": e.lanes, "rows": e.rows, "column": e.column,
             "tile": e.tile, "pairs": int(e.pairs), "cells": int(e.cells), "ms": float(e.ms),
             "launch": e.launch, "family_hi": e.family_hi, "family_lo": e.family_lo,
             "family_waves": e.family_waves} for e in arr[:n.value]]


def _i32(n):
    return (ctypes.c_int32 * max(1, n))()


def sw_shapes(h: int):
    """Compiled sweep shapes: list of (precision, lanes, rows)."""
    lib = load_library()
    n = ctypes.c_int(0)
    lib.sw_shapes(h, None, None, None, 0, ctypes.byref(n))
    p, w, r = _i32(n.value), _i32(n.value), _i32(n.value)
    _check(h, lib.sw_shapes(h, p, w, r, n.value, ctypes.byref(n)))
    return [(p[k], w[k], r[k]) for k in range(n.value)]


def sw_set_routing(h: int, precision: int, table):
    """table: list of (rows_max, lanes, rows); [] restores the default."""
    n = len(table)
    hi, w, r = _i32(n), _i32(n), _i32(n)
    for k, (a, b, c) in enumerate(table):
        hi[k], w[k], r[k] = int(a), int(b), int(c)
    _check(h, load_library().sw_set_routing(h, precision, hi, w, r, n))


def sw_get_routing(h: int, precision: int):
    lib = load_library()
    n = ctypes.c_int(0)
    lib.sw_get_routing(h, precision, None, None, None, 0, ctypes.byref(n))
    hi, w, r = _i32(n.value), _i32(n.value), _i32(n.value)
    _check(h, lib.sw_get_routing(h, precision, hi, w, r, n.value, ctypes.byref(n)))
    return [(hi[k], w[k], r[k]) for k in range(n.value)]


def routing_string(precision: int, table) -> str:
    """The tuning-string form of a routing table (sw_create's "route16=")."""
    return "route%d=" % precision + "/".join("%dx%d@%d" % (w, r, hi) for hi, w, r in table)


# ---- torch-facing helpers ----------------------------------------------------

RESULT_FIELDS = ("score", "q_start", "q_end", "r_start", "r_end")


class DeviceBatch:
    """A batch resident in device memory as torch tensors."""

    def __init__(self, queries, q_off, refs, r_off, scheme_id, schemes):
        self.queries = queries
        self.q_off = q_off
        self.refs = refs
        self.r_off = r_off
        self.scheme_id = scheme_id
        self.schemes = list(schemes)

    @property
    def n_pairs(self) -> int:
        return int(self.q_off.numel() - 1)

    @staticmethod
    def from_host(batch, device="cuda:0") -> "DeviceBatch":
        import torch
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        q = batch.queries if batch.queries.size else np.zeros(1, np.uint8)
        r = batch.refs if batch.refs.size else np.zeros(1, np.uint8)
        return DeviceBatch(t(q, torch.uint8), t(batch.q_off, torch.int64), t(r, torch.uint8),
                           t(batch.r_off, torch.int64), t(batch.scheme_id, torch.uint8), batch.schemes)

    def c_struct(self) -> sw_batch:
        b = sw_batch()
        b.queries = self.queries.data_ptr()
        b.q_off = self.q_off.data_ptr()
        b.refs = self.refs.data_ptr()
        b.r_off = self.r_off.data_ptr()
        b.scheme_id = self.scheme_id.data_ptr() if self.scheme_id is not None else None
        b.n_pairs = self.n_pairs
        return b


def make_schemes(schemes: Sequence) -> "tuple":
    """Host-side sw_scheme array (keeps the matrices alive in the tuple)."""
    arr = (sw_scheme * max(1, len(schemes)))()
    keep = []
    for k, s in enumerate(schemes):
        m = np.ascontiguousarray(s.matrix, dtype=np.int8)
        keep.append(m)
        arr[k].matrix = m.ctypes.data
        arr[k].alphabet = int(m.shape[0])
        arr[k].gap_open = int(s.gap_open)
        arr[k].gap_extend = int(s.gap_extend)
    return arr, keep


class Aligner:
    """Owns one sw_handle on one device."""

    def __init__(self, device: int = 0, tuning: Optional[str] = None, **options):
        self.device = device
        self.h = sw_create(device, tuning)
        for k, v in options.items():
            sw_set_option(self.h, k, v)

    def close(self):
        if self.h:
            sw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, key, value):
        sw_set_option(self.h, key, value)

    def get_option(self, key):
        return sw_get_option(self.h, key)

    def align(self, dbatch: DeviceBatch, out=None, stream=None):
        """Align a DeviceBatch; returns an int32 tensor [n_pairs, 5] on the
        device (score, q_start, q_end, r_start, r_end)."""
        import torch
        dev = dbatch.q_off.device
        if out is None:
            out = torch.empty((dbatch.n_pairs, 5), dtype=torch.int32, device=dev)
        assert out.is_contiguous() and out.dtype == torch.int32 and out.shape == (dbatch.n_pairs, 5)
        arr, keep = make_schemes(dbatch.schemes)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        rc = sw_align_batch(self.h, dbatch.c_struct(), arr, len(dbatch.schemes),
                            out.data_ptr() if dbatch.n_pairs else None, ctypes.c_void_p(s.cuda_stream))
        _check(self.h, rc)
        del keep
        return out

    def submit(self, dbatch: DeviceBatch, out, stream=None) -> int:
        """Enqueue the alignment of a DeviceBatch into `out` (int32 [n_pairs,
        5] on the device) without waiting; returns the ticket for poll().
        The batch and `out` are kept referenced until the ticket is polled."""
        import torch
        assert out.is_contiguous() and out.dtype == torch.int32 and out.shape == (dbatch.n_pairs, 5)
        arr, keep = make_schemes(dbatch.schemes)
        s = stream if stream is not None else torch.cuda.current_stream(dbatch.q_off.device)
        rc, t = sw_submit(self.h, dbatch.c_struct(), arr, len(dbatch.schemes),
                          out.data_ptr() if dbatch.n_pairs else None, ctypes.c_void_p(s.cuda_stream))
        _check(self.h, rc)
        del keep
        self._inflight = getattr(self, "_inflight", {})
        self._inflight[t] = (dbatch, out)
        return t

    def poll(self, ticket: int, wait: bool = True) -> bool:
        """True once the call of `ticket` has finished (raises SwError if it
        failed), False while it runs (wait=False only)."""
        rc = sw_poll(self.h, ticket, 1 if wait else 0)
        if rc == SW_PENDING:
            return False
        getattr(self, "_inflight", {}).pop(ticket, None)
        _check(self.h, rc)
        return True

    def align_noalloc(self, dbatch: DeviceBatch, out, stream=None):
        """align() through sw_align_batch_noalloc: the caller provides `out`
        (int32 [n_pairs, 5] on the device); the library allocates nothing."""
        import torch
        assert out.is_contiguous() and out.dtype == torch.int32 and out.shape == (dbatch.n_pairs, 5)
        arr, keep = make_schemes(dbatch.schemes)
        s = stream if stream is not None else torch.cuda.current_stream(dbatch.q_off.device)
        rc = sw_align_batch_noalloc(self.h, dbatch.c_struct(), arr, len(dbatch.schemes),
                                    out.data_ptr() if dbatch.n_pairs else None, ctypes.c_void_p(s.cuda_stream))
        _check(self.h, rc)
        del keep
        return out

    def align_cigar(self, dbatch: DeviceBatch, out=None, cigar_off=None, cigar=None, cigar_len=None, stream=None):
        """Align a DeviceBatch and recover every pair's path.  Returns (out,
        cigar_off, cigar, cigar_len) on the device: results as for align();
        pair i's runs ((length << 4) | SAM op code) are
        cigar[cigar_off[i] : cigar_off[i] + cigar_len[i]].  By default each
        pair gets room for q_len + r_len runs, which always suffices."""
        import torch
        dev = dbatch.q_off.device
        n = dbatch.n_pairs
        if out is None:
            out = torch.empty((n, 5), dtype=torch.int32, device=dev)
        if cigar_off is None:
            room = (dbatch.q_off[1:] - dbatch.q_off[:-1]) + (dbatch.r_off[1:] - dbatch.r_off[:-1])
            cigar_off = torch.zeros(n + 1, dtype=torch.int64, device=dev)
            if n:
                torch.cumsum(room, 0, out=cigar_off[1:])
        if cigar is None:
            cigar = torch.empty(max(1, int(cigar_off[-1].item())), dtype=torch.int32, device=dev)
        if cigar_len is None:
            cigar_len = torch.empty(max(1, n), dtype=torch.int32, device=dev)
        assert out.is_contiguous() and out.dtype == torch.int32 and out.shape == (n, 5)
        assert cigar_off.is_contiguous() and cigar_off.dtype == torch.int64 and cigar_off.numel() == n + 1
        assert cigar.is_contiguous() and cigar.dtype in (torch.int32, torch.uint32)
        assert cigar_len.is_contiguous() and cigar_len.dtype == torch.int32 and cigar_len.numel() >= n
        arr, keep = make_schemes(dbatch.schemes)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        rc = sw_align_cigar(self.h, dbatch.c_struct(), arr, len(dbatch.schemes),
                            out.data_ptr() if n else None, cigar_off.data_ptr(), cigar.data_ptr(),
                            cigar_len.data_ptr(), ctypes.c_void_p(s.cuda_stream))
        _check(self.h, rc)
        del keep
        return out, cigar_off, cigar, cigar_len

    def search(self, query, refs, r_off, scheme, out=None, stream=None):
        """Align one query (a uint8 device tensor) against every reference
        (refs: uint8 device tensor, r_off: int64 device tensor [n+1]) with one
        scheme; returns an int32 tensor [n, 5] on the device."""
        import torch
        n = int(r_off.numel()) - 1
        if out is None:
            out = torch.empty((n, 5), dtype=torch.int32, device=r_off.device)
        assert out.is_contiguous() and out.dtype == torch.int32 and out.shape == (n, 5)
        for t in (query, refs):
            assert t.dtype == torch.uint8 and t.is_contiguous()
        assert r_off.dtype == torch.int64 and r_off.is_contiguous()
        arr, keep = make_schemes([scheme])
        s = stream if stream is not None else torch.cuda.current_stream(r_off.device)
        rc = load_library().sw_search(self.h, query.data_ptr() if query.numel() else None, int(query.numel()),
                                      refs.data_ptr() if refs.numel() else None, r_off.data_ptr(), n, arr,
                                      out.data_ptr() if n else None, ctypes.c_void_p(s.cuda_stream))
        _check(self.h, rc)
        del keep
        return out

    def cigar_stats(self):
        return sw_last_cigar_stats(self.h)

    def stats(self):
        return sw_last_stats(self.h)

    def timing(self):
        return sw_last_timing(self.h)

    def bin_stats(self):
        return sw_last_bin_stats(self.h)

    def host_timing(self):
        """(enqueue_ms, wait_ms) of the last call, host wall time."""
        a, b = ctypes.c_double(0), ctypes.c_double(0)
        _check(self.h, load_library().sw_last_host_timing(self.h, ctypes.byref(a), ctypes.byref(b)))
        return float(a.value), float(b.value)

    def shapes(self):
        return sw_shapes(self.h)

    def set_routing(self, precision: int, table):
        sw_set_routing(self.h, precision, table)

    def routing(self, precision: int):
        return sw_get_routing(self.h, precision)


class Server:
    """Continuous-batching alignment server (sw_server_*).  Requests are
    workloads.Batch objects (host arrays); results come back as int32
    arrays [n_pairs, 5]."""

    def __init__(self, schemes, device: int = 0, pool_bytes: int = 16 << 30, slots: int = 3,
                 max_batch_pairs: int = 1 << 20, tuning: Optional[str] = None):
        lib = load_library()
        self._arr, self._keep = make_schemes(schemes)
        self.n_schemes = len(schemes)
        self.s = lib.sw_server_create(device, self._arr, len(schemes), int(pool_bytes), int(slots),
                                      int(max_batch_pairs), tuning.encode() if tuning else None)
        if not self.s:
            raise RuntimeError("sw_server_create failed")

    def close(self):
        if self.s:
            load_library().sw_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self):
        return load_library().sw_server_last_error(self.s).decode(errors="replace")

    def submit(self, batch) -> int:
        """Queue a workloads.Batch whose scheme ids index this server's schemes."""
        lib = load_library()
        q = np.ascontiguousarray(batch.queries, np.uint8)
        r = np.ascontiguousarray(batch.refs, np.uint8)
        qo = np.ascontiguousarray(batch.q_off, np.int64)
        ro = np.ascontiguousarray(batch.r_off, np.int64)
        sid = np.ascontiguousarray(batch.scheme_id, np.uint8)
        t = ctypes.c_uint64(0)
        rc = lib.sw_server_submit(self.s, q.ctypes.data if q.size else None, qo.ctypes.data,
                                  r.ctypes.data if r.size else None, ro.ctypes.data,
                                  sid.ctypes.data if sid.size else None, batch.n_pairs, ctypes.byref(t))
        if rc != SW_OK:
            raise SwError(rc, self._err())
        self._sizes = getattr(self, "_sizes", {})
        self._sizes[int(t.value)] = batch.n_pairs
        return int(t.value)

    def poll(self, ticket: int, wait: bool = True):
        """(results int32 [n, 5], latency_ms) or None if still pending."""
        n = self._sizes.get(ticket, 0)
        out = np.zeros((max(n, 1), 5), np.int32)
        lat = ctypes.c_double(0)
        rc = load_library().sw_server_poll(self.s, ticket, out.ctypes.data, 1 if wait else 0, ctypes.byref(lat))
        if rc == SW_PENDING:
            return None
        self._sizes.pop(ticket, None)
        if rc != SW_OK:
            raise SwError(rc, self._err())
        return out[:n], float(lat.value)

    def timing(self):
        """Cumulative ms spent admitting, aligning and fetching."""
        vals = [ctypes.c_double(0) for _ in range(3)]
        load_library().sw_server_timing(self.s, *[ctypes.byref(v) for v in vals])
        return {k: float(v.value) for k, v in zip(("admit_ms", "align_ms", "fetch_ms"), vals)}

    def stats(self):
        vals = [ctypes.c_int64(0) for _ in range(5)]
        load_library().sw_server_stats(self.s, *[ctypes.byref(v) for v in vals])
        keys = ("pool_peak_bytes", "pool_capacity", "requests_done", "batches", "pairs_done")
        return {k: int(v.value) for k, v in zip(keys, vals)}
