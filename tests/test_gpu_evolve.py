"""The evolutionary parameter search on the GPU, at a tiny budget: every
configuration it accepts reproduces the default results (checked inside the
fitness function), and the best one still matches the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_12350_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_search_and_analysis_on_the_gpu():
    import torch
    from paper_2208_12350_amd import evolve as E
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch
    b = W.make_workload("dna_large", n_pairs=4000)
    db = DeviceBatch.from_host(b)
    fit = E.LibraryFitness(db, repeats=1)
    ev = E.Evaluator(fit)
    best, best_ms, hist, ev = E.evolve(ev, fit.shapes, population=6, generations=2, seed=3, weights=fit.weights)
    assert hist == sorted(hist, reverse=True)
    assert best_ms <= ev([]) + 1e-9
    # an invalid configuration fails instead of running
    assert ev([("route", 0, 2048, 16, 1)]) is None
    rep = E.analyse(best, ev)
    assert set(map(tuple, rep["weak"] + rep["strong"])) == set(map(tuple, best))
    # the chosen configuration aligns exactly like the oracle
    cfg = E.apply_edits(fit.default_route, best, fit.shapes)
    al = Aligner(0, E.tuning_string(*cfg))
    out = al.align(db).cpu().numpy()
    al.close()
    idx = np.arange(0, b.n_pairs, 13)
    ora = O.align_batch(b, index=idx)
    want = np.stack([ora[f] for f in ("score", "q_start", "q_end", "r_start", "r_end")], axis=1)
    assert np.array_equal(out[idx], want)
