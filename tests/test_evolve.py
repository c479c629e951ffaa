"""CPU tests of the evolutionary parameter search and the edit analysis
(Algorithms 1 and 2) against synthetic fitness functions whose structure
(independent, weak and interacting edits) is known."""
import random

import pytest

from paper_2208_12350_amd import evolve as E

SHAPES = [(16, r) for r in range(1, 17)] + [(32, r) for r in range(9, 17)] + [(64, r) for r in range(9, 33)]
DEFAULT = [(16, k + 1) if k < 16 else (32, 16) if k < 32 else (64, 32) for k in range(128)]


def test_apply_edits_and_tuning_string():
    cfg = E.apply_edits(DEFAULT, [("route", 0, 64, 16, 4), ("opt", "streams", 2)], SHAPES)
    route, opts = cfg
    assert route[:4] == [(16, 4)] * 4 and route[4] == DEFAULT[4]
    assert opts == {"streams": 2}
    s = E.tuning_string(route, opts)
    assert s.startswith("route16=16x4@64/16x5@80/") and s.endswith(";streams=2")
    # a later edit overrides an earlier one where they overlap
    route2, _ = E.apply_edits(DEFAULT, [("route", 0, 64, 16, 4), ("route", 32, 48, 16, 8)], SHAPES)
    assert route2[2] == (16, 8) and route2[3] == (16, 4)
    # invalid: shape too small for its rows, unknown shape, bad option value
    assert E.apply_edits(DEFAULT, [("route", 0, 128, 16, 4)], SHAPES) is None
    assert E.apply_edits(DEFAULT, [("route", 0, 16, 8, 2)], SHAPES) is None
    assert E.apply_edits(DEFAULT, [("opt", "streams", 9)], SHAPES) is None


def test_random_edits_and_operators_are_well_formed():
    rng = random.Random(3)
    g = []
    for _ in range(200):
        g = E.mutate(g, rng, SHAPES)
        for e in g:
            assert e[0] in ("route", "opt")
            if e[0] == "route":
                assert 0 <= e[1] < e[2] <= 2048 and e[1] % 16 == 0 and e[2] % 16 == 0
                assert (e[3], e[4]) in SHAPES and e[3] * e[4] >= e[1] + 16
    a, b = [1, 2, 3], [4, 5]
    for _ in range(20):
        c, d = E.crossover(a, b, rng)
        assert sorted(c + d) == sorted(a + b)


# A synthetic program: time 10 ms times a factor per edit present.
#   e1: 0.90 alone and in any context        (independent)
#   e2: 0.995                                  (weak)
#   e3: 1.0                                    (weak: a no-op)
#   e4 needs e5: e4 without e5 fails; together 0.80; e5 alone 1.0  (epistatic pair)
E1, E2, E3, E4, E5 = [("opt", "k%d" % i, 1) for i in range(1, 6)]


def synthetic(edits):
    s = set(edits)
    if E4 in s and E5 not in s:
        return None
    t = 10.0
    if E1 in s:
        t *= 0.90
    if E2 in s:
        t *= 0.995
    if E4 in s and E5 in s:
        t *= 0.80
    return t


def test_weak_edits_algorithm_1():
    edits = [E2, E1, E4, E3, E5]
    weaks = E.weak_edits(edits, synthetic)
    assert weaks == [E2, E3]


def test_independent_and_epistatic_algorithm_2():
    strong = [E1, E4, E5]
    indep, epi, savings = E.split_independent(strong, synthetic)
    assert indep == [E1]
    assert epi == [E4, E5]


def test_analyse_end_to_end():
    rep = E.analyse([E2, E1, E4, E3, E5], synthetic)
    assert rep["weak"] == [E2, E3] and rep["independent"] == [E1] and rep["epistatic"] == [E4, E5]
    sub = dict(rep["epistatic_subsets"])
    assert sub[0] == 10.0 and sub[1] is None and sub[2] == 10.0 and sub[3] == pytest.approx(8.0)
    assert rep["t_all"] == pytest.approx(10 * 0.9 * 0.995 * 0.8)


def test_evolution_improves_and_keeps_its_best():
    # routing edits: the best route for bucket 0 is 16x1 and for bucket 1
    # 16x2 (5% each, independent); colpath=0 costs 20%; the workload's
    # queries all fall in buckets 0-1, and the search is told so
    def measure(edits):
        cfg = E.apply_edits(default, edits, shapes)
        if cfg is None:
            return None
        route, opts = cfg
        t = 10.0
        t *= 0.95 if route[0] == (16, 1) else 1.0
        t *= 0.95 if route[1] == (16, 2) else 1.0
        if opts.get("colpath", 1) == 0:
            t *= 1.2
        return t
    shapes = [(16, 1), (16, 2), (16, 4), (16, 8), (32, 16), (64, 32)]
    default = [(16, 8)] * 8 + [(32, 16)] * 24 + [(64, 32)] * 96
    weights = [100, 100] + [0.01] * 126
    found = 0
    for seed in range(4):
        best, best_ms, hist, ev = E.evolve(measure, shapes, population=24, generations=20, seed=seed,
                                           weights=weights, max_span=2)
        assert hist == sorted(hist, reverse=True)          # elitism: the best never gets worse
        assert hist[-1] == best_ms == measure(best)
        assert best_ms < 10.0
        found += best_ms <= 10.0 * 0.95 * 0.95 + 1e-9
        # the analysis recovers the two route edits as the strong, independent ones
        if best_ms <= 10.0 * 0.95 * 0.95 + 1e-9:
            rep = E.analyse(best, measure)
            assert len(rep["independent"]) == 2 and not rep["epistatic"]
            assert rep["t_strong"] == pytest.approx(best_ms)
    assert found >= 2


def test_evaluator_shares_measurements_of_equal_configurations():
    calls = []

    class M:
        def key(self, edits):
            cfg = E.apply_edits(DEFAULT, edits, SHAPES)
            return "fail" if cfg is None else E.tuning_string(cfg[0], {k: v for k, v in cfg[1].items() if v != 4})

        def __call__(self, edits):
            calls.append(list(edits))
            return 1.0

    ev = E.Evaluator(M())
    ev([])
    ev([("opt", "streams", 4)])                  # the default value: same configuration
    ev([("route", 0, 16, 16, 1)])                # the default shape of bucket 0: same configuration
    ev([("route", 0, 16, 16, 2)])                # a different configuration
    assert len(calls) == 2 and ev.calls == 2
