"""The autotuner on the GPU: rates come from real probe launches, and the
routing it picks aligns every pair exactly as the oracle does."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_12350_amd import workloads as W

pytestmark = pytest.mark.gpu
FIELDS = ("score", "q_start", "q_end", "r_start", "r_end")


def test_autotuned_routing_is_exact():
    import torch
    from paper_2208_12350_amd import autotune as T
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch, routing_string
    shapes = [(16, 2), (16, 4), (16, 8), (16, 16), (32, 8), (32, 16), (64, 9), (64, 16), (64, 32)]
    rates = T.measure_rates(0, 16, m=256, target_cells=2e8, repeats=1, shapes=shapes)
    assert set(rates) == set(shapes) and all(v > 0 for v in rates.values())
    b = W.make_workload("mixed", n_pairs=1200, seed=8181)
    table = T.choose_routing(b.q_len(), b.r_len(), rates)
    assert {(w, r) for _, w, r in table} <= set(shapes)
    al = Aligner(0, routing_string(16, table))
    try:
        assert al.routing(16) == table
        out = al.align(DeviceBatch.from_host(b))
        want = O.align_batch(b)
        assert np.array_equal(out.cpu().numpy(), np.stack([want[f] for f in FIELDS], axis=1))
    finally:
        al.close()
