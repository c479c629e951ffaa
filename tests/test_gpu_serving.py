"""GPU tests of the continuous-batching server: results of each request are
bit-identical alone and in a mix of concurrently submitted requests; the
admission budget is never exceeded; bad requests are rejected at submit."""
import threading
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_12350_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("score", "q_start", "q_end", "r_start", "r_end")


def _requests(k, seed, lo=20, hi=400):
    rng = np.random.default_rng(seed)
    # one protein scheme for every request (a server holds one scheme set)
    return [W.make_workload("mixed", n_pairs=int(rng.integers(lo, hi)), seed=seed * 100 + i, scheme_seed=seed)
            for i in range(k)]


def _alone(reqs):
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch
    al = Aligner(0)
    try:
        return [al.align(DeviceBatch.from_host(b)).cpu().numpy() for b in reqs]
    finally:
        al.close()


def test_mix_equals_alone_and_oracle():
    from paper_2208_12350_amd.binding import Server
    reqs = _requests(24, 31)
    want = _alone(reqs)
    srv = Server(reqs[0].schemes, slots=3, pool_bytes=256 << 20, max_batch_pairs=4000)
    try:
        tickets = [None] * len(reqs)
        rng = np.random.default_rng(5)

        def producer():
            for i, b in enumerate(reqs):
                tickets[i] = srv.submit(b)
                time.sleep(float(rng.exponential(0.002)))

        th = threading.Thread(target=producer)
        th.start()
        th.join()
        lat = []
        for i, b in enumerate(reqs):
            got, ms = srv.poll(tickets[i], wait=True)
            assert np.array_equal(got, want[i]), i
            lat.append(ms)
        st = srv.stats()
        assert st["requests_done"] == len(reqs)
        assert st["pairs_done"] == sum(b.n_pairs for b in reqs)
        assert st["batches"] <= len(reqs)
    finally:
        srv.close()
    # the alone results themselves agree with the oracle on a sample
    for i in (0, 7, 19):
        o = O.align_batch(reqs[i])
        assert np.array_equal(want[i], np.stack([o[f] for f in FIELDS], axis=1))


def test_small_pool_budget_is_respected():
    from paper_2208_12350_amd.binding import Server
    reqs = _requests(12, 77, 200, 600)
    need = [int(b.queries.size + b.refs.size + 33 * b.n_pairs) for b in reqs]
    cap = 3 * max(need) + (1 << 16)     # room for about three requests at once
    want = _alone(reqs)
    srv = Server(reqs[0].schemes, slots=2, pool_bytes=cap, max_batch_pairs=2000)
    try:
        ts = [srv.submit(b) for b in reqs]   # burst: most must wait for admission
        for i, t in enumerate(ts):
            got, _ = srv.poll(t, wait=True)
            assert np.array_equal(got, want[i]), i
        st = srv.stats()
        assert 0 < st["pool_peak_bytes"] <= st["pool_capacity"] <= cap
        assert st["requests_done"] == len(reqs)
    finally:
        srv.close()


def test_bad_requests_rejected_at_submit():
    from paper_2208_12350_amd.binding import Server, SwError, SW_EINVAL, SW_ENOMEM, SW_ETOOLONG
    dna = W.dna_scheme()
    srv = Server([dna], slots=1, pool_bytes=1 << 20, max_batch_pairs=1000)
    try:
        bad = W.from_pairs([(np.array([0, 9], np.uint8), np.array([1, 2], np.uint8))], [0], [dna])
        with pytest.raises(SwError) as e:
            srv.submit(bad)
        assert e.value.code == SW_EINVAL
        long_q = W.from_pairs([(np.zeros(3000, np.uint8), np.zeros(5, np.uint8))], [0], [dna])
        with pytest.raises(SwError) as e:
            srv.submit(long_q)
        assert e.value.code == SW_ETOOLONG
        huge = W.from_pairs([(np.zeros(2000, np.uint8), np.zeros(60000, np.uint8))] * 30, [0] * 30, [dna])
        with pytest.raises(SwError) as e:
            srv.submit(huge)
        assert e.value.code == SW_ENOMEM
        ok = W.make_workload("dna_small", n_pairs=10)
        t = srv.submit(ok)
        got, _ = srv.poll(t, wait=True)
        o = O.align_batch(ok)
        assert np.array_equal(got, np.stack([o[f] for f in FIELDS], axis=1))
    finally:
        srv.close()
