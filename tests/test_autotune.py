"""Host logic of the routing autotuner (no GPU): the choice minimises the
predicted time, covers every query length, and round-trips through the
table form the library accepts."""
import numpy as np
import pytest

from paper_2208_12350_amd import autotune as T
from paper_2208_12350_amd import workloads as W

SHAPES16 = ([(16, r) for r in range(1, 17)] + [(32, r) for r in range(5, 17)] + [(64, r) for r in range(9, 33)]
            + [(256, r) for r in range(3, 9)])


def _valid(table):
    prev = 0
    for hi, w, r in table:
        assert hi > prev and hi % 16 == 0 and w * r >= hi
        prev = hi
    assert prev == 2048


def test_uniform_rates_pick_fewest_slots():
    rates = {s: 1.0 for s in SHAPES16}
    rng = np.random.default_rng(0)
    q = rng.integers(1, 2049, size=5000)
    r = rng.integers(1, 3000, size=5000)
    table = T.choose_routing(q, r, rates)
    _valid(table)
    shapes = T.expand(table)
    for k, (w, rr) in enumerate(shapes):
        rows = 16 * (k + 1)
        # with equal rates the narrowest covering tile of each width wins,
        # and among widths the one with the fewest slots for that bucket
        m = r[(np.minimum(q, 2048) - 1) // 16 == k]
        m = m if m.size else np.array([max(512.0, 2.0 * rows + 64)])
        best = min((s for s in SHAPES16 if s[0] * s[1] >= rows),
                   key=lambda s: (float(np.sum(T.slots(m, s))), s[0] * s[1]))
        assert (w, rr) == best


def test_faster_shape_family_wins():
    rates = {s: 1.0 for s in SHAPES16}
    for s in SHAPES16:
        if s[0] == 32:
            rates[s] = 3.0          # 32-lane groups three times faster
    q = np.array([300, 400, 500, 20, 1500])
    r = np.array([700, 900, 1000, 50, 3000])
    shapes = T.expand(T.choose_routing(q, r, rates))
    assert shapes[(300 - 1) // 16][0] == 32
    assert shapes[(500 - 1) // 16][0] == 32
    assert shapes[(1500 - 1) // 16][0] == 64        # no 32-lane shape covers 1500 rows


def test_tuned_table_is_never_predicted_slower():
    rng = np.random.default_rng(1)
    rates = {s: float(rng.uniform(0.5, 2.0)) for s in SHAPES16}
    b = W.make_workload("mixed", n_pairs=20000, seed=3)
    q, r = b.q_len(), b.r_len()
    tuned = T.choose_routing(q, r, rates)
    _valid(tuned)
    t_tuned = T.predicted_ms(q, r, tuned, rates)
    # any other valid table: e.g. the widest shape everywhere, or a random one
    widest = [(2048, 64, 32)]
    assert t_tuned <= T.predicted_ms(q, r, widest, rates) + 1e-9
    for trial in range(20):
        choice = []
        for k in range(128):
            rows = 16 * (k + 1)
            cover = [s for s in SHAPES16 if s[0] * s[1] >= rows]
            choice.append(cover[rng.integers(len(cover))])
        other = T.merge(choice)
        _valid(other)
        assert t_tuned <= T.predicted_ms(q, r, other, rates) + 1e-9


def test_merge_expand_round_trip_and_string():
    from paper_2208_12350_amd.binding import routing_string
    choice = [(16, 1)] * 1 + [(16, 4)] * 3 + [(32, 8)] * 12 + [(64, 32)] * 112
    table = T.merge(choice)
    assert table == [(16, 16, 1), (64, 16, 4), (256, 32, 8), (2048, 64, 32)]
    assert T.expand(table) == choice
    assert routing_string(16, table) == "route16=16x1@16/16x4@64/32x8@256/64x32@2048"


def test_no_covering_shape_is_an_error():
    with pytest.raises(ValueError):
        T.choose_routing(np.array([100]), np.array([200]), {(16, 4): 1.0})


def test_wide_group_variants():
    rates = {s: 1.0 for s in SHAPES16}
    q = np.array([100, 300, 700, 1500, 2048])
    r = np.array([200, 600, 1500, 3000, 4000])
    cands = T.candidate_tables(q, r, rates, SHAPES16)
    assert "model" in cands
    for name, table in cands.items():
        _valid(table)
        base_name = name.split("+")[0]
        if base_name.startswith("coarse"):
            step = int(base_name[len("coarse"):])
            assert base_name in cands
            # the coarse routings use rows per lane that are multiples of the step
            for w, rr in T.expand(cands[base_name]):
                assert w > 64 or rr % step == 0 or (w == 16 and rr < step)
        if "+coop>" not in name:
            continue
        above = int(name.split(">")[1])
        for k, (w, rr) in enumerate(T.expand(table)):
            rows = 16 * (k + 1)
            if rows > above:
                assert w == 256 and 256 * rr >= rows and 256 * (rr - 1) < max(rows, 256 * 3)
            else:
                assert (w, rr) == T.expand(cands[base_name])[k]
    # no cooperative shapes compiled: no cooperative variants
    only = [s for s in SHAPES16 if s[0] != 256]
    assert not any("coop" in n for n in T.candidate_tables(q, r, {s: 1.0 for s in only}, only))


def test_dominant_scheme_and_builtin_candidate():
    b = W.make_workload("mixed", n_pairs=3000, seed=11)
    assert T.dominant_scheme(b).name == "dna"                 # 80% of the pairs
    p = W.make_workload("protein", n_pairs=200, seed=12)
    assert T.dominant_scheme(p).name == "protein"
    rates = {s: 1.0 for s in SHAPES16}
    q, r = b.q_len(), b.r_len()
    builtin = [(256, 16, 16), (512, 32, 16), (2048, 256, 8)]
    cands = T.candidate_tables(q, r, rates, SHAPES16, builtin=builtin)
    assert cands["builtin"] == builtin
    assert "builtin" not in T.candidate_tables(q, r, rates, SHAPES16, builtin=cands["model"])
