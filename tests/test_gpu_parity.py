"""GPU parity: the HIP path against the CPU oracle, bit-exact on every field.

Small cases are compared on every pair; the full-size workloads (the same
launch configuration the benchmark times) are compared on a seeded sample of
pairs, which the oracle recomputes one by one, and on properties that hold
for every pair."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_12350_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("score", "q_start", "q_end", "r_start", "r_end")


@pytest.fixture(scope="module")
def aligner():
    import torch
    from paper_2208_12350_amd.binding import Aligner
    assert torch.cuda.is_available()
    a = Aligner(0)
    yield a
    a.close()


def run_gpu(aligner, batch):
    from paper_2208_12350_amd.binding import DeviceBatch
    db = DeviceBatch.from_host(batch)
    out = aligner.align(db)
    return out.cpu().numpy()


def as_tuples(o):
    return np.stack([o[f] for f in FIELDS], axis=1).astype(np.int64)


def assert_same(gpu, ora, batch, idx=None):
    ora_t = as_tuples(ora)
    g = gpu if idx is None else gpu[idx]
    bad = np.flatnonzero(np.any(g != ora_t, axis=1))
    if bad.size:
        k = int(bad[0])
        i = k if idx is None else int(idx[k])
        q, r, s = batch.pair(i)
        raise AssertionError("pair %d (n=%d m=%d scheme=%s): gpu %s oracle %s; %d mismatches"
                             % (i, q.size, r.size, s.name, g[k].tolist(), ora_t[k].tolist(), bad.size))


def test_hand_cases(aligner):
    dna = W.dna_scheme()
    pairs = [("AAAATTTT", "CAAAAGGTTTTC"), ("AC", "ACGAC"), ("AGAC", "ATAC"), ("AAAA", "CCCC"),
             ("A", "A"), ("ACGT", "ACGT"), ("GGGACGTGGG", "TTACGTTT")]
    b = W.from_pairs([(W.encode(x, "ACGT"), W.encode(y, "ACGT")) for x, y in pairs], [0] * len(pairs), [dna])
    assert_same(run_gpu(aligner, b), O.align_batch(b), b)


def test_tiny_random_all_gap_settings(aligner):
    rng = np.random.default_rng(42)
    for o, e in [(6, 1), (11, 1), (1, 1), (3, 0), (5, 2)]:
        M = rng.integers(-4, 4, size=(6, 6))
        np.fill_diagonal(M, rng.integers(1, 6, size=6))
        sc = W.Scheme(np.ascontiguousarray(M.astype(np.int8)), o, e)
        pairs = [(rng.integers(0, 6, size=int(rng.integers(0, 9))), rng.integers(0, 6, size=int(rng.integers(0, 12))))
                 for _ in range(3000)]
        b = W.from_pairs(pairs, [0] * len(pairs), [sc])
        assert_same(run_gpu(aligner, b), O.align_batch(b), b)


def test_dna_small_every_pair(aligner):
    b = W.make_workload("dna_small")
    assert_same(run_gpu(aligner, b), O.align_batch(b), b)


EDGE_Q = [1, 2, 15, 16, 17, 31, 32, 33, 100, 255, 256, 257, 383, 384, 385, 511, 512, 513, 1023, 1024, 1025, 2047, 2048]
EDGE_R = [1, 2, 15, 16, 17, 63, 64, 65, 127, 128, 129, 130, 131, 255, 256, 257, 1000, 6144]


@pytest.mark.parametrize("alphabet", ["dna", "protein"])
def test_edge_lengths(aligner, alphabet):
    """Every (query, reference) length of the grid below, up to the longest
    queries (2048) against the longest references (6144) of the mixed
    workload, half of them holding an exact copy of the query; plus mutated
    embeddings at the largest shapes (the long tail of the mixed workload)."""
    rng = np.random.default_rng(7 if alphabet == "dna" else 8)
    sc = W.dna_scheme() if alphabet == "dna" else W.protein_scheme(5)
    A = sc.alphabet
    pairs = []
    for n in EDGE_Q:
        for m in EDGE_R:
            q = rng.integers(0, A, size=n)
            if m >= n and rng.random() < 0.5:
                off = int(rng.integers(0, m - n + 1))
                r = rng.integers(0, A, size=m)
                r[off:off + n] = q
            else:
                r = rng.integers(0, A, size=m)
            pairs.append((q, r))
    for n, m in ((2048, 6144), (2048, 3072), (1024, 6144), (2048, 2048), (1500, 4500)):
        q = rng.integers(0, A, size=n)
        r = rng.integers(0, A, size=m)
        mut = q.copy()
        flip = rng.random(n) < (0.1 if A == 4 else 0.3)
        mut[flip] = (mut[flip] + rng.integers(1, A, size=int(flip.sum()))) % A
        off = int(rng.integers(0, m - n + 1))
        r[off:off + n] = mut
        pairs.append((q, r))
    b = W.from_pairs(pairs, [0] * len(pairs), [sc])
    assert_same(run_gpu(aligner, b), O.align_batch(b), b)


def test_large_gap_costs(aligner):
    """Gap costs beyond 16 bits: pairs still take the packed path (their score
    bound fits), whose operands hold each cost in a 16-bit half; any cost of
    0x7C00 or more must act exactly as the true cost (no gap can ever pay)."""
    rng = np.random.default_rng(31)
    dna = W.dna_scheme()
    schemes = [W.Scheme(dna.matrix, o, e, "dna_o%d_e%d" % (o, e))
               for o, e in ((65537, 1), (70000, 70000), (2000, 1), (40000, 3))]
    pairs, sids = [], []
    for k in range(2000):
        n = int(rng.integers(1, 300))
        q = rng.integers(0, 4, size=n).astype(np.uint8)
        mut = q.copy()
        flip = rng.random(n) < 0.1
        mut[flip] = (mut[flip] + 1) % 4
        if rng.random() < 0.3:
            cut = int(rng.integers(0, n))
            mut = np.concatenate([mut[:cut], rng.integers(0, 4, size=int(rng.integers(1, 4))).astype(np.uint8),
                                  mut[cut:]])
        r = np.concatenate([rng.integers(0, 4, size=int(rng.integers(0, 80))), mut,
                            rng.integers(0, 4, size=int(rng.integers(0, 80)))]).astype(np.uint8)
        pairs.append((q, r))
        sids.append(k % len(schemes))
    b = W.from_pairs(pairs, sids, schemes)
    g = run_gpu(aligner, b)
    assert aligner.stats()[2] == 0          # every pair took the packed path
    assert_same(g, O.align_batch(b), b)


def test_many_items_per_wave_64_lane_groups(aligner):
    """Regression: queries of 257-1024 rows run on 64-lane groups; with many
    more work items than resident wavefronts every wavefront loops over
    several items (a lane-0-only fetch at the head of that loop was once
    lowered into an inner loop that never fetched again)."""
    rng = np.random.default_rng(12)
    dna = W.dna_scheme()
    pairs = []
    for _ in range(6000):
        n = int(rng.integers(257, 700))
        q = rng.integers(0, 4, size=n)
        r = np.concatenate([rng.integers(0, 4, size=int(rng.integers(0, 50))), q,
                            rng.integers(0, 4, size=int(rng.integers(0, 50)))])
        pairs.append((q, r))
    b = W.from_pairs(pairs, [0] * len(pairs), [dna])
    g = run_gpu(aligner, b)
    idx = np.arange(0, b.n_pairs, 13)
    assert_same(g, O.align_batch(b, index=idx), b, idx=idx)


def test_all_mismatch_and_empty(aligner):
    dna = W.dna_scheme()
    pairs = [(np.zeros(50, np.uint8), np.ones(70, np.uint8)), (np.zeros(0, np.uint8), np.ones(7, np.uint8)),
             (np.ones(9, np.uint8), np.zeros(0, np.uint8)), (np.zeros(0, np.uint8), np.zeros(0, np.uint8)),
             (np.full(300, 2, np.uint8), np.full(500, 2, np.uint8))]
    b = W.from_pairs(pairs, [0] * len(pairs), [dna])
    assert_same(run_gpu(aligner, b), O.align_batch(b), b)


def test_protein_sample(aligner):
    b = W.make_workload("protein", n_pairs=1500)
    assert_same(run_gpu(aligner, b), O.align_batch(b), b)


def test_mixed_sample_two_schemes(aligner):
    b = W.make_workload("mixed", n_pairs=3000)
    assert_same(run_gpu(aligner, b), O.align_batch(b), b)


def test_max_query_bound():
    """The max_query option leaves the bins above the bound unlaunched:
    the results are the oracle's, the same with the option and without,
    and a batch with a longer query is rejected (SW_ETOOLONG), after which
    the handle works again."""
    from paper_2208_12350_amd.binding import Aligner, SwError, SW_ETOOLONG
    b = W.make_workload("protein", n_pairs=2000, seed=41)
    longest = int(b.q_len().max())
    plain = Aligner(0)
    bound = Aligner(0, max_query=longest)
    try:
        assert bound.get_option("max_query") == longest
        g = run_gpu(plain, b)
        assert_same(g, O.align_batch(b), b)
        assert np.array_equal(run_gpu(bound, b), g)
        bound.set_option("max_query", longest - 1)
        with pytest.raises(SwError) as ei:
            run_gpu(bound, b)
        assert ei.value.code == SW_ETOOLONG
        bound.set_option("max_query", 0)
        assert np.array_equal(run_gpu(bound, b), g)
        with pytest.raises(SwError):
            bound.set_option("max_query", 2049)
    finally:
        plain.close()
        bound.close()


def test_repeatable_and_order_invariant(aligner):
    b = W.make_workload("dna_small", n_pairs=700, seed=99)
    g1 = run_gpu(aligner, b)
    g2 = run_gpu(aligner, b)
    assert np.array_equal(g1, g2)
    perm = np.random.default_rng(3).permutation(b.n_pairs)
    gp = run_gpu(aligner, b.subset(perm))
    assert np.array_equal(gp, g1[perm])


def test_invalid_inputs_are_rejected(aligner):
    from paper_2208_12350_amd.binding import SwError, SW_EINVAL, SW_ETOOLONG
    dna = W.dna_scheme()
    bad = W.from_pairs([(np.array([0, 1, 7], np.uint8), np.array([0, 1, 2], np.uint8))], [0], [dna])
    with pytest.raises(SwError) as ei:
        run_gpu(aligner, bad)
    assert ei.value.code == SW_EINVAL
    long_q = W.from_pairs([(np.zeros(2049, np.uint8), np.zeros(10, np.uint8))], [0], [dna])
    with pytest.raises(SwError) as ei:
        run_gpu(aligner, long_q)
    assert ei.value.code == SW_ETOOLONG
    bad_sid = W.from_pairs([(np.zeros(5, np.uint8), np.zeros(5, np.uint8))], [1], [dna])
    with pytest.raises(SwError) as ei:
        run_gpu(aligner, bad_sid)
    assert ei.value.code == SW_EINVAL
    # the handle still works after errors
    ok = W.make_workload("dna_small", n_pairs=20)
    assert_same(run_gpu(aligner, ok), O.align_batch(ok), ok)


@pytest.mark.timeout(600)
def test_mixed_full_size_tuned_routing():
    """The mixed workload at full size (1,000,000 DNA and protein pairs) with
    the routing the benchmark times: every candidate routing of the
    autotuner gives the same bits on every pair, a seeded sample of pairs
    matches the oracle, and every pair satisfies the result properties."""
    import torch
    from paper_2208_12350_amd import autotune as T
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch, routing_string
    b = W.make_workload("mixed")
    db = DeviceBatch.from_host(b)
    name, table, cands, tile = T.tune_batch(b, db, 0, repeats=2)
    out = torch.empty((b.n_pairs, 5), dtype=torch.int32, device="cuda:0")
    al = Aligner(0, T.tuning_string(table, tile))
    try:
        al.align(db, out)
        al.align(db, out)          # a graph replay, as timed
        g = out.cpu().numpy()
        assert al.stats()[2] == 0
    finally:
        al.close()
    for other, t in cands.items():
        if other == name:
            continue
        alo = Aligner(0, T.tuning_string(t, 64 if tile == 128 else 128))
        try:
            out.fill_(-7)
            alo.align(db, out)
            assert np.array_equal(out.cpu().numpy(), g), other
        finally:
            alo.close()
    rng = np.random.default_rng(13)
    idx = np.sort(rng.choice(b.n_pairs, size=1500, replace=False))
    # plus the longest queries, which run on the widest shapes
    idx = np.union1d(idx, np.argsort(b.q_len())[-200:])
    assert_same(g, O.align_batch(b, index=idx), b, idx=idx)
    ql, rl = b.q_len(), b.r_len()
    assert np.all(g[:, 0] > 0)
    assert np.all((g[:, 1] >= 0) & (g[:, 1] <= g[:, 2]) & (g[:, 2] < ql))
    assert np.all((g[:, 3] >= 0) & (g[:, 3] <= g[:, 4]) & (g[:, 4] < rl))


@pytest.mark.parametrize("name", ["dna_large", "protein"])
def test_full_size_sampled(aligner, name):
    b = W.make_workload(name)
    g = run_gpu(aligner, b)
    idx = np.sort(np.random.default_rng(11).choice(b.n_pairs, size=1500, replace=False))
    assert_same(g, O.align_batch(b, index=idx), b, idx=idx)
    # properties of every pair
    ql, rl = b.q_len(), b.r_len()
    s = g[:, 0]
    assert np.all(s > 0)  # every pair embeds a mutated copy of its query
    assert np.all((g[:, 1] >= 0) & (g[:, 1] <= g[:, 2]) & (g[:, 2] < ql))
    assert np.all((g[:, 3] >= 0) & (g[:, 3] <= g[:, 4]) & (g[:, 4] < rl))


def test_int16_and_int32_paths_agree(aligner):
    """The packed int16 path and the int32 path give identical results."""
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch
    b = W.make_workload("mixed", n_pairs=2000, seed=777)
    db = DeviceBatch.from_host(b)
    g16 = aligner.align(db).cpu().numpy()
    assert aligner.stats()[2] == 0          # everything fit the int16 path
    a32 = Aligner(0, precision=32)
    try:
        g32 = a32.align(db).cpu().numpy()
        assert a32.stats()[2] == b.n_pairs  # everything forced onto int32
    finally:
        a32.close()
    assert np.array_equal(g16, g32)
    idx = np.arange(0, b.n_pairs, 7)
    assert_same(g16, O.align_batch(b, index=idx), b, idx=idx)


def test_large_scores_route_to_int32(aligner):
    """A scheme whose scores would overflow 16 bits runs on the int32 path,
    side by side with int16 pairs of another scheme in the same batch; the
    scaled scheme gives exactly k times the score and the same coordinates."""
    base = W.make_workload("dna_small", n_pairs=300, seed=5)
    k = 40
    dna = W.dna_scheme()
    big = W.Scheme(np.ascontiguousarray((dna.matrix.astype(np.int32) * k).astype(np.int8)),
                   dna.gap_open * k, dna.gap_extend * k, "dna_x40")
    pairs = [base.pair(i)[:2] for i in range(base.n_pairs)]
    # long pairs so that min(n, m) * 120 exceeds the int16 bound
    rng = np.random.default_rng(8)
    for _ in range(50):
        q = rng.integers(0, 4, size=int(rng.integers(300, 700))).astype(np.uint8)
        r = np.concatenate([rng.integers(0, 4, size=50), q, rng.integers(0, 4, size=80)]).astype(np.uint8)
        pairs.append((q, r))
    sids = [i % 2 for i in range(len(pairs))]
    b = W.from_pairs(pairs, sids, [dna, big])
    g = run_gpu(aligner, b)
    assert aligner.stats()[2] > 0           # some pairs took the int32 path
    assert_same(g, O.align_batch(b), b)
    b1 = W.from_pairs(pairs, [0] * len(pairs), [dna])
    g1 = run_gpu(aligner, b1)
    odd = np.arange(1, len(pairs), 2)
    assert np.array_equal(g[odd, 0], g1[odd, 0] * k)
    assert np.array_equal(g[odd, 1:], g1[odd, 1:])


def test_plain_persistent_and_graph_modes_agree():
    """Plain per-bin launches, persistent launches and graph replays give the
    same bits.  The captured graph is replayed several times, with other
    eager GPU work and host synchronisation in between, and every replay is
    checked (graphs must not depend on state left by an earlier replay)."""
    import torch
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch
    b = W.make_workload("mixed", n_pairs=2500, seed=4242)
    db = DeviceBatch.from_host(b)
    want = O.align_batch(b)
    want = np.stack([want[f] for f in FIELDS], axis=1)
    results = {}
    for name, opts in (("plain", dict(mode=0, graph=0)), ("persistent", dict(mode=1, graph=0)),
                       ("graph", dict(mode=1, graph=1))):
        al = Aligner(0, **opts)
        try:
            out = torch.full((b.n_pairs, 5), -7, dtype=torch.int32, device="cuda:0")
            for rep in range(4 if name == "graph" else 1):
                out.fill_(-7)
                al.align(db, out)
                got = out.cpu().numpy()
                assert np.array_equal(got, want), (name, rep)
                # unrelated eager work between replays
                x = torch.randn(1 << 20, device="cuda:0")
                torch.cuda.synchronize()
                assert float(x.abs().sum()) > 0
            results[name] = al.stats()
        finally:
            al.close()
    assert results["plain"] == results["persistent"] == results["graph"]


@pytest.mark.gpu
def test_streams_and_per_launch_timing_agree():
    """Persistent launches over 1..4 streams and the serialised per-launch
    timing mode give the same bits; per-launch statistics add up to the
    call's totals (cells per pass, one pair per non-trivial pair)."""
    import torch
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch
    b = W.make_workload("mixed", n_pairs=1800, seed=5151)
    db = DeviceBatch.from_host(b)
    want = O.align_batch(b)
    want_arr = np.stack([want[f] for f in FIELDS], axis=1)
    nontrivial = int(np.sum((b.q_len() > 0) & (b.r_len() > 0)))
    positive = int(np.sum(want["score"] > 0))
    for opts in (dict(streams=1), dict(streams=2), dict(streams=4), dict(timing=2),
                 dict(timing=2, families=0), dict(mode=0, graph=0, timing=2)):
        al = Aligner(0, **opts)
        try:
            out = torch.full((b.n_pairs, 5), -7, dtype=torch.int32, device="cuda:0")
            al.align(db, out)
            assert np.array_equal(out.cpu().numpy(), want_arr), opts
            fwd, rev, _ = al.stats()
            st = al.bin_stats()
            assert sum(e["cells"] for e in st if e["pass"] == 0) == fwd
            assert sum(e["cells"] for e in st if e["pass"] == 1) == rev
            assert sum(e["pairs"] for e in st if e["pass"] == 0) == nontrivial
            assert sum(e["pairs"] for e in st if e["pass"] == 1) == positive
            if opts.get("timing") == 2:
                # every (pass, shape) with pairs ran at least one of its kernels
                by_bin = {}
                for e in st:
                    k = (e["pass"], e["precision"], e["lanes"], e["rows"])
                    p_, m_ = by_bin.get(k, (0, 0.0))
                    by_bin[k] = (p_ + e["pairs"], m_ + e["ms"])
                assert all(m > 0 for p, m in by_bin.values() if p > 0), opts
                # the bins of one launch share its time; family launches
                # exactly when persistent mode has families on
                launches = {}
                for e in st:
                    if e["launch"] >= 0:
                        launches.setdefault((e["pass"], e["launch"]), set()).add((e["ms"], e["family_hi"],
                                                                                 e["family_lo"]))
                assert all(len(v) == 1 for v in launches.values()), opts
                fam = any(e["family_hi"] > 0 for e in st)
                assert fam == (opts.get("families", 1) == 1 and opts.get("mode", 1) == 1), opts
            else:
                assert all(e["ms"] == 0 for e in st)
        finally:
            al.close()


def _routing(widths):
    """A routing table that, for each 16-row bucket, uses the first listed
    group width whose compiled shapes cover it, with the smallest R."""
    R_OF = {16: range(1, 17), 32: range(5, 17), 64: range(9, 33), 256: range(3, 9)}
    table = []
    for hi in range(16, 2049, 16):
        for w in widths:
            rs = [r for r in R_OF[w] if w * r >= hi]
            if rs:
                table.append((hi, w, rs[0]))
                break
    return table


@pytest.mark.gpu
def test_routing_choices_agree():
    """Results never depend on which shape sweeps a pair: 16-, 32- and
    64-lane routings all reproduce the oracle."""
    import torch
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch
    b = W.make_workload("mixed", n_pairs=1500, seed=6161)
    db = DeviceBatch.from_host(b)
    want = O.align_batch(b)
    want_arr = np.stack([want[f] for f in FIELDS], axis=1)
    al = Aligner(0)
    try:
        default = al.routing(16)
        assert default[-1][0] == 2048
        for widths in ((64,), (32, 64), (16, 32, 64), (16, 64), (256,), (16, 32, 256)):
            al.set_routing(16, _routing(widths))
            got_table = al.routing(16)
            assert got_table[-1][0] == 2048
            out = torch.full((b.n_pairs, 5), -7, dtype=torch.int32, device="cuda:0")
            al.align(db, out)
            assert np.array_equal(out.cpu().numpy(), want_arr), widths
            used = {(e["lanes"], e["rows"]) for e in al.bin_stats() if e["pairs"] > 0 and e["precision"] == 16}
            assert {w for w, _ in used} <= set(widths), (widths, used)
        al.set_routing(16, [])
        assert al.routing(16) == default
    finally:
        al.close()


@pytest.mark.gpu
def test_routing_rejects_bad_tables():
    from paper_2208_12350_amd.binding import Aligner, SwError
    al = Aligner(0)
    try:
        before = al.routing(16)
        for bad in ([(2048, 16, 16)],                       # 256 rows cannot cover 2048
                    [(1024, 64, 16), (512, 64, 32)],         # rows_max decreasing
                    [(1000, 64, 16), (2048, 64, 32)],        # not a multiple of 16
                    [(1024, 64, 16)],                        # does not reach 2048
                    [(2048, 64, 33)],                        # not compiled
                    [(2048, 48, 48)]):                       # not compiled
            with pytest.raises(SwError):
                al.set_routing(16, bad)
            assert al.routing(16) == before
        with pytest.raises(SwError):
            al.set_routing(8, [(2048, 64, 32)])
    finally:
        al.close()


@pytest.mark.gpu
def test_int16_range_edges(aligner):
    """Pairs at the edges of the packed path's range: int8 extreme scores
    (+127 / -128, gap open 127) with min(n, m) * 127 just below and just
    above the int16 bound, and references just below and above the packed
    path's length limit.  Every pair must match the oracle, and exactly the
    pairs beyond a bound take the int32 path."""
    A = 4
    mat = np.full((A, A), -128, dtype=np.int8)
    np.fill_diagonal(mat, 127)
    ext = W.Scheme(np.ascontiguousarray(mat), 127, 1, "extreme")
    rng = np.random.default_rng(99)
    lim_n = 30592 // 127                     # 240: the longest query on the packed path
    pairs, expect_i32 = [], 0
    for n in (lim_n - 1, lim_n, lim_n + 1, lim_n + 2):
        q = rng.integers(0, A, size=n).astype(np.uint8)
        pairs.append((q, q.copy()))                                   # self-alignment: S = 127 n
        r = np.concatenate([rng.integers(0, A, size=30), q, rng.integers(0, A, size=17)]).astype(np.uint8)
        pairs.append((q, r))
        expect_i32 += 2 if n > lim_n else 0
    for m in (31999, 32000, 32001, 40000, 60000):
        q = rng.integers(0, A, size=60).astype(np.uint8)
        r = rng.integers(0, A, size=m).astype(np.uint8)
        r[m // 3:m // 3 + 60] = q
        pairs.append((q, r))
        expect_i32 += 1 if m > 32000 else 0
    b = W.from_pairs(pairs, [0] * len(pairs), [ext])
    g = run_gpu(aligner, b)
    assert aligner.stats()[2] == expect_i32
    want = O.align_batch(b)
    assert_same(g, want, b)
    assert g[0, 0] == 127 * (lim_n - 1) and g[2, 0] == 127 * lim_n


@pytest.mark.gpu
def test_graph_replays_across_batch_sizes():
    """One captured graph serves batches of different sizes on the same
    buffers: the batch size is read on the device at every replay, so pairs
    beyond it are never touched and every prefix matches the oracle."""
    import torch
    from paper_2208_12350_amd.binding import (Aligner, DeviceBatch, make_schemes, sw_align_batch,
                                              sw_get_option)
    b = W.make_workload("mixed", n_pairs=3000, seed=9191)
    db = DeviceBatch.from_host(b)
    want = O.align_batch(b)
    want = np.stack([want[f] for f in FIELDS], axis=1)
    al = Aligner(0, capacity=3000)
    arr, keep = make_schemes(db.schemes)
    out = torch.empty((b.n_pairs, 5), dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream()
    try:
        for n in (3000, 1200, 1, 2999, 1200, 0, 3000):
            out.fill_(-7)
            cb = db.c_struct()
            cb.n_pairs = n
            rc = sw_align_batch(al.h, cb, arr, len(db.schemes), out.data_ptr(), ctypes.c_void_p(stream.cuda_stream))
            assert rc == 0, al.h
            got = out.cpu().numpy()
            assert np.array_equal(got[:n], want[:n]), n
            assert (got[n:] == -7).all(), n
            x = torch.randn(1 << 18, device="cuda:0")        # unrelated eager work between replays
            assert float(x.abs().sum()) > 0
        assert sw_get_option(al.h, "captures") == 1
    finally:
        al.close()


@pytest.mark.gpu
def test_column_word_and_table_paths_agree():
    """Small-alphabet pairs read their scores from per-column words (option
    colpath); the table-lookup path gives the same bits, on a mix of schemes
    that can and cannot take the column path."""
    import torch
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch
    rng = np.random.default_rng(4321)
    dna = W.dna_scheme()
    m3 = np.array([[2, -1, -2], [-1, 3, -1], [-2, -1, 1]], dtype=np.int8)     # 3 letters: column path
    tri = W.Scheme(np.ascontiguousarray(m3), 4, 2, "tri")
    wide = W.Scheme(np.ascontiguousarray(dna.matrix), 300, 2, "dna_o300")     # M + o > 255: table path
    prot = W.protein_scheme(5)                                                 # 20 letters: table path
    schemes = [dna, tri, wide, prot]
    pairs, sids = [], []
    for k in range(1600):
        s = int(rng.integers(0, 4))
        A = schemes[s].alphabet
        n = int(rng.integers(1, 300))
        q = rng.integers(0, A, size=n).astype(np.uint8)
        r = np.concatenate([rng.integers(0, A, size=int(rng.integers(0, 60))), q,
                            rng.integers(0, A, size=int(rng.integers(0, 200)))]).astype(np.uint8)
        if rng.random() < 0.3:
            r = rng.integers(0, A, size=int(rng.integers(1, 400))).astype(np.uint8)
        pairs.append((q, r))
        sids.append(s)
    b = W.from_pairs(pairs, sids, schemes)
    db = DeviceBatch.from_host(b)
    want = O.align_batch(b)
    want = np.stack([want[f] for f in FIELDS], axis=1)
    outs = {}
    for colpath in (1, 0):
        al = Aligner(0, colpath=colpath, timing=2)
        try:
            out = al.align(db).cpu().numpy()
            assert np.array_equal(out, want), colpath
            col_pairs = sum(e["pairs"] for e in al.bin_stats() if e["column"] == 1)
            if colpath:
                assert col_pairs > 0
            else:
                assert col_pairs == 0
        finally:
            al.close()


@pytest.mark.parametrize("name", ["dna_large", "protein", "mixed"])
def test_narrow_tile_is_exact(name):
    """16- and 32-lane shapes streaming the reference in tiles of 64 steps
    (option chunk = 64): the same bits as the default tile on every pair, and
    the oracle's on a sample, with references around the tile boundaries."""
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch
    b = W.make_workload(name, n_pairs=5000, seed=4040)
    rng = np.random.default_rng(41)
    sc = b.schemes[0] if name != "protein" else b.schemes[0]
    A = sc.alphabet
    pairs = [(rng.integers(0, A, size=int(n)).astype(np.uint8), rng.integers(0, A, size=int(m)).astype(np.uint8))
             for n in (1, 17, 100, 255, 300, 511) for m in (1, 2, 49, 50, 63, 64, 65, 66, 127, 128, 129, 130, 192, 193)]
    edge = W.from_pairs(pairs, [0] * len(pairs), [sc])
    for batch in (b, edge):
        db = DeviceBatch.from_host(batch)
        outs = []
        for chunk in (128, 64):
            al = Aligner(0, chunk=chunk)
            try:
                outs.append(al.align(db).cpu().numpy())
                assert al.get_option("chunk") == chunk
            finally:
                al.close()
        assert np.array_equal(outs[0], outs[1])
        idx = np.arange(batch.n_pairs) if batch is edge else np.sort(rng.choice(batch.n_pairs, 600, replace=False))
        assert_same(outs[1], O.align_batch(batch, index=idx), batch, idx=idx)
