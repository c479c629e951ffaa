"""The allocation-free entry point (sw_align_batch_noalloc) through the C ABI:
bit-identical to sw_align_batch on the same inputs, on consecutive calls
whose second batch is smaller (the static workspace keeps the first call's
contents), from two handles and in both launch modes; oversize batches are
rejected before anything is launched."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_12350_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("score", "q_start", "q_end", "r_start", "r_end")


def _oracle_rows(batch, idx=None):
    o = O.align_batch(batch, index=idx) if idx is not None else O.align_batch(batch)
    return np.stack([o[f] for f in FIELDS], axis=1).astype(np.int64)


def test_noalloc_matches_align_batch_on_consecutive_calls():
    import torch
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch
    big = W.make_workload("mixed", n_pairs=20000, seed=4242)
    small = W.make_workload("mixed", n_pairs=3000, seed=4343)
    dbig, dsmall = DeviceBatch.from_host(big), DeviceBatch.from_host(small)
    print("noalloc: mixed %d then %d pairs" % (big.n_pairs, small.n_pairs), flush=True)
    for mode in (1, 0):
        al = Aligner(0, mode=mode)
        try:
            na_big = torch.full((big.n_pairs, 5), -7, dtype=torch.int32, device="cuda:0")
            na_small = torch.full((small.n_pairs, 5), -7, dtype=torch.int32, device="cuda:0")
            al.align_noalloc(dbig, na_big)
            stats_big = al.stats()
            al.align_noalloc(dsmall, na_small)
            stats_small = al.stats()
            ref_big = al.align(dbig).cpu().numpy()
            assert al.stats() == stats_big
            ref_small = al.align(dsmall).cpu().numpy()
            assert al.stats() == stats_small
        finally:
            al.close()
        assert np.array_equal(na_big.cpu().numpy(), ref_big), "mode %d, first call" % mode
        assert np.array_equal(na_small.cpu().numpy(), ref_small), "mode %d, second call" % mode
    # and the smaller batch against the oracle on every pair
    assert np.array_equal(ref_small.astype(np.int64), _oracle_rows(small))


def test_noalloc_second_handle_and_repeat():
    """A second handle on the same device uses the same array; a repeat of
    the same batch after a larger one gives the same bits."""
    import torch
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch
    b = W.make_workload("dna_small")
    db = DeviceBatch.from_host(b)
    a1, a2 = Aligner(0), Aligner(0)
    try:
        o1 = torch.empty((b.n_pairs, 5), dtype=torch.int32, device="cuda:0")
        o2 = torch.empty((b.n_pairs, 5), dtype=torch.int32, device="cuda:0")
        a1.align_noalloc(db, o1)
        a2.align_noalloc(db, o2)
        # neither handle has reserved per-pair workspace of its own
        assert a1.get_option("capacity") == 0 and a2.get_option("capacity") == 0
        ref = a1.align(db).cpu().numpy()
        assert a1.get_option("capacity") >= b.n_pairs
    finally:
        a1.close()
        a2.close()
    assert np.array_equal(o1.cpu().numpy(), ref)
    assert np.array_equal(o2.cpu().numpy(), ref)
    assert np.array_equal(ref.astype(np.int64), _oracle_rows(b))


def test_noalloc_rejects_oversize_batch():
    """More pairs than the static workspace holds: SW_EINVAL from the host
    check, before any pointer is read or any kernel launched."""
    import torch
    from paper_2208_12350_amd import binding as B
    al = B.Aligner(0)
    try:
        dummy = torch.zeros(16, dtype=torch.int64, device="cuda:0")
        bs = B.sw_batch()
        bs.queries = bs.q_off = bs.refs = bs.r_off = dummy.data_ptr()
        bs.scheme_id = None
        bs.n_pairs = B.SW_NOALLOC_MAX_PAIRS + 1
        arr, keep = B.make_schemes([W.dna_scheme()])
        rc = B.sw_align_batch_noalloc(al.h, bs, arr, 1, dummy.data_ptr(), None)
        assert rc == B.SW_EINVAL
        assert "at most" in B.sw_last_error(al.h)
        # the handle still works afterwards
        b = W.make_workload("dna_small", n_pairs=200)
        db = B.DeviceBatch.from_host(b)
        out = torch.empty((b.n_pairs, 5), dtype=torch.int32, device="cuda:0")
        al.align_noalloc(db, out)
        assert np.array_equal(out.cpu().numpy().astype(np.int64), _oracle_rows(b))
    finally:
        al.close()
