"""ctypes wrapper around the scalar C oracle (sw_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this module; the GPU library never imports it and it
never imports the GPU library.  See sw_oracle.c for what is computed.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_sw.so")
CFLAGS = ["-O2", "-std=c99", "-shared", "-fPIC", "-pthread"]


class _Scheme(ctypes.Structure):
    _fields_ = [("matrix", ctypes.c_void_p), ("alphabet", ctypes.c_int32),
                ("gap_open", ctypes.c_int32), ("gap_extend", ctypes.c_int32)]


RESULT_DTYPE = np.dtype([("score", np.int32), ("q_start", np.int32), ("q_end", np.int32),
                         ("r_start", np.int32), ("r_end", np.int32)])


def build(force: bool = True) -> str:
    """Compile the oracle into liboracle_sw.so next to its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + CFLAGS + ["-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_align_batch.restype = ctypes.c_int
        lib.oracle_align_batch.argtypes = [ctypes.c_void_p] * 5 + [ctypes.c_int64, ctypes.c_void_p,
                                                                    ctypes.c_int, ctypes.c_void_p,
                                                                    ctypes.c_int64, ctypes.c_void_p,
                                                                    ctypes.c_int]
        lib.oracle_align_pair.restype = ctypes.c_int
        lib.oracle_align_pair.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_cigar_pair.restype = ctypes.c_int
        lib.oracle_cigar_pair.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p]
        lib.oracle_cigar_batch.restype = ctypes.c_int
        lib.oracle_cigar_batch.argtypes = [ctypes.c_void_p] * 5 + [ctypes.c_int64, ctypes.c_void_p,
                                                                    ctypes.c_int, ctypes.c_void_p,
                                                                    ctypes.c_int64] + [ctypes.c_void_p] * 4 + [
                                                                    ctypes.c_int]
        lib.oracle_score_matrix.restype = ctypes.c_int
        lib.oracle_score_matrix.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def _schemes_array(schemes):
    keep = []
    arr = (_Scheme * max(1, len(schemes)))()
    for k, s in enumerate(schemes):
        mat = np.ascontiguousarray(s.matrix, dtype=np.int8)
        keep.append(mat)
        arr[k].matrix = mat.ctypes.data
        arr[k].alphabet = mat.shape[0]
        arr[k].gap_open = int(s.gap_open)
        arr[k].gap_extend = int(s.gap_extend)
    return arr, keep


def _ptr(x: np.ndarray):
    return x.ctypes.data if x.size else None


def align_batch(batch, index: Optional[Sequence[int]] = None, threads: Optional[int] = None) -> np.ndarray:
    """Align all pairs of a workloads.Batch (or the subset ``index``) and
    return a structured array with fields score, q_start, q_end, r_start,
    r_end."""
    lib = _load()
    queries = np.ascontiguousarray(batch.queries, dtype=np.uint8)
    refs = np.ascontiguousarray(batch.refs, dtype=np.uint8)
    q_off = np.ascontiguousarray(batch.q_off, dtype=np.int64)
    r_off = np.ascontiguousarray(batch.r_off, dtype=np.int64)
    sid = np.ascontiguousarray(batch.scheme_id, dtype=np.uint8)
    arr, keep = _schemes_array(batch.schemes)
    if index is None:
        idx = None
        n_out = batch.n_pairs
    else:
        idx = np.ascontiguousarray(np.asarray(index, dtype=np.int64))
        n_out = idx.size
    out = np.zeros(n_out, dtype=RESULT_DTYPE)
    if n_out == 0:
        return out
    threads = threads or os.cpu_count() or 1
    rc = lib.oracle_align_batch(_ptr(queries), q_off.ctypes.data, _ptr(refs), r_off.ctypes.data,
                                sid.ctypes.data, batch.n_pairs, ctypes.addressof(arr), len(batch.schemes),
                                None if idx is None else idx.ctypes.data, 0 if idx is None else idx.size,
                                out.ctypes.data, int(threads))
    if rc != 0:
        raise ValueError("oracle: invalid input (residue outside alphabet or bad offsets)")
    del keep
    return out


def align_pair(a, b, scheme):
    """Align one pair; returns (score, q_start, q_end, r_start, r_end)."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    arr, keep = _schemes_array([scheme])
    out = np.zeros(1, dtype=RESULT_DTYPE)
    rc = lib.oracle_align_pair(_ptr(a), a.size, _ptr(b), b.size, ctypes.addressof(arr), out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle: invalid input")
    del keep
    r = out[0]
    return (int(r["score"]), int(r["q_start"]), int(r["q_end"]), int(r["r_start"]), int(r["r_end"]))


def score_matrix(a, b, scheme) -> np.ndarray:
    """The full (n+1) x (m+1) H matrix of the forward pass."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    arr, keep = _schemes_array([scheme])
    H = np.zeros((a.size + 1, b.size + 1), dtype=np.int64)
    rc = lib.oracle_score_matrix(_ptr(a), a.size, _ptr(b), b.size, ctypes.addressof(arr), H.ctypes.data)
    if rc != 0:
        raise ValueError("oracle: allocation failure")
    del keep
    return H


# SAM/BAM operation codes of the runs ((length << 4) | op)
OP_I, OP_D, OP_EQ, OP_X = 1, 2, 7, 8
_OP_CHAR = {OP_I: "I", OP_D: "D", OP_EQ: "=", OP_X: "X"}


def cigar_string(runs) -> str:
    """Runs ((length << 4) | op) -> text such as '4=1I5='."""
    return "".join("%d%s" % (int(r) >> 4, _OP_CHAR[int(r) & 15]) for r in runs)


def cigar_pair(a, b, scheme):
    """Result and alignment path of one pair: ((score, q_start, q_end,
    r_start, r_end), runs as a uint32 array)."""
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    arr, keep = _schemes_array([scheme])
    res = np.zeros(1, dtype=RESULT_DTYPE)
    if lib.oracle_align_pair(_ptr(a), a.size, _ptr(b), b.size, ctypes.addressof(arr), res.ctypes.data) != 0:
        raise ValueError("oracle: invalid input")
    runs = np.zeros(max(1, a.size + b.size), dtype=np.uint32)
    n = ctypes.c_int64(0)
    if lib.oracle_cigar_pair(_ptr(a), a.size, _ptr(b), b.size, ctypes.addressof(arr), res.ctypes.data,
                             runs.ctypes.data, runs.size, ctypes.byref(n)) != 0:
        raise ValueError("oracle: traceback failed")
    del keep
    r = res[0]
    return ((int(r["score"]), int(r["q_start"]), int(r["q_end"]), int(r["r_start"]), int(r["r_end"])),
            runs[:n.value].copy())


def cigar_batch(batch, index: Optional[Sequence[int]] = None, threads: Optional[int] = None,
                results: Optional[np.ndarray] = None):
    """Results and alignment paths of all pairs of a workloads.Batch (or of
    the subset ``index``).  Returns (results, runs, run_off, n_runs): the
    runs of the k-th pair are runs[run_off[k] : run_off[k] + n_runs[k]].
    ``results`` (of the same pairs, in the same order) skips the alignment."""
    lib = _load()
    res = align_batch(batch, index=index, threads=threads) if results is None else \
        np.ascontiguousarray(results, dtype=RESULT_DTYPE)
    queries = np.ascontiguousarray(batch.queries, dtype=np.uint8)
    refs = np.ascontiguousarray(batch.refs, dtype=np.uint8)
    q_off = np.ascontiguousarray(batch.q_off, dtype=np.int64)
    r_off = np.ascontiguousarray(batch.r_off, dtype=np.int64)
    sid = np.ascontiguousarray(batch.scheme_id, dtype=np.uint8)
    idx = None if index is None else np.ascontiguousarray(np.asarray(index, dtype=np.int64))
    pairs = np.arange(batch.n_pairs) if idx is None else idx
    cap = (q_off[pairs + 1] - q_off[pairs]) + (r_off[pairs + 1] - r_off[pairs])
    run_off = np.zeros(pairs.size + 1, dtype=np.int64)
    np.cumsum(cap, out=run_off[1:])
    runs = np.zeros(max(1, int(run_off[-1])), dtype=np.uint32)
    n_runs = np.zeros(pairs.size, dtype=np.int64)
    if pairs.size:
        arr, keep = _schemes_array(batch.schemes)
        rc = lib.oracle_cigar_batch(_ptr(queries), q_off.ctypes.data, _ptr(refs), r_off.ctypes.data,
                                    sid.ctypes.data, batch.n_pairs, ctypes.addressof(arr), len(batch.schemes),
                                    None if idx is None else idx.ctypes.data, 0 if idx is None else idx.size,
                                    res.ctypes.data, run_off.ctypes.data, runs.ctypes.data, n_runs.ctypes.data,
                                    int(threads or os.cpu_count() or 1))
        del keep
        if rc != 0:
            raise ValueError("oracle: traceback failed")
    return res, runs, run_off, n_runs
