"""GPU parity of the alignment paths (sw_align_cigar) against the oracle's
traceback: the runs of every compared pair must be identical, and the
results must equal the score path's.  Small cases are compared on every
pair; the full-size DNA workload on a seeded sample, and on properties that
hold for every pair (the runs consume exactly the result box)."""
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


def gpu_paths(aligner, batch, **kw):
    """(results [n, 5], runs uint32, cigar_off, cigar_len) on the host."""
    from paper_2208_12350_amd.binding import DeviceBatch
    db = DeviceBatch.from_host(batch)
    out, off, cig, ln = aligner.align_cigar(db, **kw)
    return (out.cpu().numpy().astype(np.int64), cig.cpu().numpy().view(np.uint32),
            off.cpu().numpy(), ln.cpu().numpy()[:batch.n_pairs])


def assert_paths_equal(batch, gpu, idx=None):
    res, runs, off, ln = gpu
    idx = np.arange(batch.n_pairs) if idx is None else np.asarray(idx)
    ores, oruns, ooff, onr = O.cigar_batch(batch, index=idx)
    want = np.stack([ores[f] for f in FIELDS], axis=1).astype(np.int64)
    bad = np.flatnonzero(np.any(res[idx] != want, axis=1))
    assert bad.size == 0, ("results differ", int(idx[bad[0]]), res[idx[bad[0]]].tolist(), want[bad[0]].tolist())
    for k, i in enumerate(idx):
        g = runs[off[i]:off[i] + ln[i]]
        o = oruns[ooff[k]:ooff[k] + onr[k]]
        if ln[i] != onr[k] or not np.array_equal(g, o):
            q, r, s = batch.pair(int(i))
            raise AssertionError("pair %d (n=%d m=%d %s) result %s: gpu %s oracle %s"
                                 % (i, q.size, r.size, s.name, res[i].tolist(), O.cigar_string(g),
                                    O.cigar_string(o)))


def _fig2():
    M = np.full((4, 4), -2, np.int8)
    np.fill_diagonal(M, 2)
    return W.Scheme(M, 1, 1, "fig2")


def test_golden_cases(aligner):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "cigar_cases.txt")
    pairs, sids, want = [], [], []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, q, r, cig = line.split()
            pairs.append((W.encode(q, "ACGT"), W.encode(r, "ACGT")))
            sids.append(0 if name == "dna" else 1)
            want.append(cig)
    b = W.from_pairs(pairs, sids, [W.dna_scheme(), _fig2()])
    res, runs, off, ln = gpu_paths(aligner, b)
    got = [O.cigar_string(runs[off[i]:off[i] + ln[i]]) or "*" for i in range(b.n_pairs)]
    assert got == want


def test_tiny_random_all_gap_settings(aligner):
    rng = np.random.default_rng(7)
    for o, e in [(6, 1), (1, 1), (3, 0), (5, 2), (2, 1)]:
        M = rng.integers(-4, 4, size=(4, 4))
        np.fill_diagonal(M, rng.integers(2, 6, size=4))
        sc = W.Scheme(np.ascontiguousarray(M.astype(np.int8)), o, e)
        pairs = [(rng.integers(0, 4, size=int(rng.integers(0, 20))), rng.integers(0, 4, size=int(rng.integers(0, 24))))
                 for _ in range(1500)]
        b = W.from_pairs(pairs, [0] * len(pairs), [sc])
        assert_paths_equal(b, gpu_paths(aligner, b))


def test_large_gap_costs(aligner):
    """Gap costs beyond 16 bits on the packed box sweep: the paths equal the
    oracle's (with such costs an optimal path has no gap, so it is one
    substitution run between the box corners)."""
    rng = np.random.default_rng(32)
    dna = W.dna_scheme()
    schemes = [W.Scheme(dna.matrix, o, e, "dna_o%d_e%d" % (o, e))
               for o, e in ((65537, 1), (70000, 70000), (2000, 1), (40000, 3))]
    pairs, sids = [], []
    for k in range(800):
        n = int(rng.integers(1, 200))
        q = rng.integers(0, 4, size=n).astype(np.uint8)
        mut = q.copy()
        flip = rng.random(n) < 0.1
        mut[flip] = (mut[flip] + 1) % 4
        if rng.random() < 0.3:
            cut = int(rng.integers(0, n))
            mut = np.concatenate([mut[:cut], rng.integers(0, 4, size=2).astype(np.uint8), mut[cut:]])
        r = np.concatenate([rng.integers(0, 4, size=int(rng.integers(0, 50))), mut,
                            rng.integers(0, 4, size=int(rng.integers(0, 50)))]).astype(np.uint8)
        pairs.append((q, r))
        sids.append(k % len(schemes))
    b = W.from_pairs(pairs, sids, schemes)
    assert_paths_equal(b, gpu_paths(aligner, b))


def test_dna_small_every_pair(aligner):
    b = W.make_workload("dna_small")
    assert_paths_equal(b, gpu_paths(aligner, b))


def test_protein_and_mixed_samples(aligner):
    for name, n in (("protein", 1500), ("mixed", 3000)):
        b = W.make_workload(name, n_pairs=n)
        gpu = gpu_paths(aligner, b)
        # every pair below 4M box cells, plus a few of the largest boxes
        res = gpu[0]
        cells = (res[:, 2] - res[:, 1] + 1) * (res[:, 4] - res[:, 3] + 1) * (res[:, 0] > 0)
        idx = np.flatnonzero(cells < 4_000_000)
        idx = np.concatenate([idx, np.argsort(cells)[-3:]])
        assert_paths_equal(b, gpu, idx)


def test_edge_shapes(aligner):
    # box heights around every shape boundary, long boxes, identical and
    # unrelated sequences, empty inputs
    rng = np.random.default_rng(11)
    dna = W.dna_scheme()
    pairs = []
    for n in (1, 2, 7, 8, 9, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 1535, 1536, 1537,
              2047, 2048):
        q = rng.integers(0, 4, size=n).astype(np.uint8)
        r = np.concatenate([rng.integers(0, 4, size=int(rng.integers(0, 40))), q,
                            rng.integers(0, 4, size=int(rng.integers(0, 40)))]).astype(np.uint8)
        pairs.append((q, r))
        mut = q.copy()
        flip = rng.random(n) < 0.1
        mut[flip] = (mut[flip] + 1) % 4
        pairs.append((mut, r))
    pairs.append((np.zeros(0, np.uint8), rng.integers(0, 4, size=10).astype(np.uint8)))
    pairs.append((rng.integers(0, 4, size=10).astype(np.uint8), np.zeros(0, np.uint8)))
    pairs.append((np.zeros(50, np.uint8), np.ones(60, np.uint8)))        # no positive cell
    pairs.append((rng.integers(0, 4, size=300).astype(np.uint8), rng.integers(0, 4, size=5000).astype(np.uint8)))
    b = W.from_pairs(pairs, [0] * len(pairs), [dna])
    assert_paths_equal(b, gpu_paths(aligner, b))


def test_results_equal_score_path(aligner):
    from paper_2208_12350_amd.binding import DeviceBatch
    b = W.make_workload("mixed", n_pairs=5000)
    db = DeviceBatch.from_host(b)
    plain = aligner.align(db).cpu().numpy()
    out, _, _, ln = aligner.align_cigar(db)
    assert np.array_equal(out.cpu().numpy(), plain)
    assert np.all((ln.cpu().numpy() > 0) == (plain[:, 0] > 0))


def _consumed(runs, off, ln, ops):
    """Per pair, the residues consumed by runs whose op is in `ops`."""
    n = ln.size
    total = np.zeros(n, np.int64)
    lens = (runs >> 4).astype(np.int64)
    take = np.isin(runs & 15, ops)
    vals = np.where(take, lens, 0)
    csum = np.concatenate([[0], np.cumsum(vals)])
    start = off[:n]
    total = csum[start + ln] - csum[start]
    return total


def test_full_size_dna_large_sampled(aligner):
    b = W.make_workload("dna_large")
    res, runs, off, ln = gpu_paths(aligner, b)
    pos = res[:, 0] > 0
    assert np.all(ln[pos] >= 1) and np.all(ln[~pos] == 0)
    # every path consumes exactly its box
    q_used = _consumed(runs, off, ln, (7, 8, 1))
    r_used = _consumed(runs, off, ln, (7, 8, 2))
    assert np.array_equal(q_used[pos], res[pos, 2] - res[pos, 1] + 1)
    assert np.array_equal(r_used[pos], res[pos, 4] - res[pos, 3] + 1)
    # first and last runs are substitution columns
    first = runs[off[:-1][pos]] & 15
    last = runs[off[:-1][pos] + ln[pos] - 1] & 15
    assert np.all(np.isin(first, (7, 8))) and np.all(np.isin(last, (7, 8)))
    idx = np.random.default_rng(3).choice(b.n_pairs, size=400, replace=False)
    assert_paths_equal(b, (res, runs, off, ln), np.sort(idx))


@pytest.mark.parametrize("name,n", [("dna_large", 20000), ("mixed", 6000)])
def test_chunked_workspace_gives_the_same_paths(aligner, name, n):
    # mixed: each chunk's bins hold column-word and table pairs, and most
    # pairs lie outside the chunk (the trivial key, left out of the order)
    from paper_2208_12350_amd.binding import Aligner
    b = W.make_workload(name, n_pairs=n)
    whole = gpu_paths(aligner, b)
    _, rec_bytes, chunks, _, _ = aligner.cigar_stats()
    assert chunks == 1
    small = Aligner(0, cigar_workspace=130_000_000)
    try:
        parts = gpu_paths(small, b)
        _, rec2, chunks2, _, _ = small.cigar_stats()
    finally:
        small.close()
    assert rec2 == rec_bytes and chunks2 >= 3, (rec2, chunks2)
    for x, y in zip(whole, parts):
        assert np.array_equal(x, y)


def test_small_room_is_reported(aligner):
    import torch
    from paper_2208_12350_amd.binding import DeviceBatch, SwError
    b = W.make_workload("dna_small", n_pairs=300)
    db = DeviceBatch.from_host(b)
    n = b.n_pairs
    off = torch.arange(n + 1, dtype=torch.int64, device="cuda:0") * 2   # room for 2 runs each
    with pytest.raises(SwError):
        aligner.align_cigar(db, cigar_off=off)
    # recompute the lengths the oracle needs
    ores, oruns, ooff, onr = O.cigar_batch(b)
    _, _, _, ln = aligner.align_cigar(DeviceBatch.from_host(b))   # a fresh, big enough room
    ln = ln.cpu().numpy()[:n]
    assert np.array_equal(ln, onr)
    # and the failing call marked exactly the pairs that need more than 2 runs
    out = torch.empty((n, 5), dtype=torch.int32, device="cuda:0")
    cig = torch.empty(2 * n, dtype=torch.int32, device="cuda:0")
    cl = torch.empty(n, dtype=torch.int32, device="cuda:0")
    with pytest.raises(SwError):
        aligner.align_cigar(db, out=out, cigar_off=off, cigar=cig, cigar_len=cl)
    cl = cl.cpu().numpy()
    assert np.array_equal(cl == -1, onr > 2)
    assert np.array_equal(cl[onr <= 2], onr[onr <= 2])


def test_int16_and_int32_path_sweeps_agree(aligner):
    # the packed int16 path sweep takes every pair whose score fits; forcing
    # int32 must give the same paths
    from paper_2208_12350_amd.binding import Aligner
    b = W.make_workload("mixed", n_pairs=4000)
    packed = gpu_paths(aligner, b)
    wide = Aligner(0, precision=32)
    try:
        plain = gpu_paths(wide, b)
    finally:
        wide.close()
    for x, y in zip(packed, plain):
        assert np.array_equal(x, y)


def test_large_scores_take_the_int32_path_sweep(aligner):
    rng = np.random.default_rng(5)
    M = np.full((4, 4), -60, np.int8)
    np.fill_diagonal(M, 100)
    sc = W.Scheme(M, 120, 20)
    pairs = []
    for n in (500, 700, 900, 1200):
        q = rng.integers(0, 4, size=n).astype(np.uint8)
        r = q.copy()
        r[rng.random(n) < 0.05] = 0
        r = np.concatenate([rng.integers(0, 4, size=30), r[: n // 2], rng.integers(0, 4, size=3), r[n // 2:]])
        pairs.append((q, r.astype(np.uint8)))
    b = W.from_pairs(pairs, [0] * len(pairs), [sc])
    gpu = gpu_paths(aligner, b)
    assert np.all(gpu[0][:, 0] > 30592)
    assert_paths_equal(b, gpu)


def test_column_word_and_table_path_sweeps_agree(aligner):
    # when every scheme of a call has at most four residues whose scores
    # plus the gap open cost fit a byte, the packed path sweep reads column
    # words; with colpath=0 every pair takes the table form, which must write
    # the same records.  In a call with one scheme outside that set, each
    # packed bin is split: its pairs of eligible schemes take column words,
    # the others the table form.
    from paper_2208_12350_amd.binding import Aligner
    rng = np.random.default_rng(21)
    M = rng.integers(-5, 1, size=(4, 4))
    np.fill_diagonal(M, rng.integers(1, 6, size=4))
    col_scheme = W.Scheme(np.ascontiguousarray(M.astype(np.int8)), 7, 2)      # M + o >= 0
    M = rng.integers(-9, 1, size=(4, 4))
    np.fill_diagonal(M, 4)
    M[0, 1] = -9
    table_scheme = W.Scheme(np.ascontiguousarray(M.astype(np.int8)), 2, 1)    # M + o < 0
    pairs = []
    for k in range(3000):
        n = int(rng.integers(1, 700))
        q = rng.integers(0, 4, size=n).astype(np.uint8)
        r = np.concatenate([rng.integers(0, 4, size=int(rng.integers(0, 60))), q,
                            rng.integers(0, 4, size=int(rng.integers(0, 60)))]).astype(np.uint8)
        flip = rng.random(r.size) < 0.08
        r[flip] = (r[flip] + 1) % 4
        pairs.append((q, r))
    batches = [W.from_pairs(pairs, [k % 2 for k in range(len(pairs))], [W.dna_scheme(), col_scheme]),
               W.from_pairs(pairs, [k % 3 for k in range(len(pairs))], [W.dna_scheme(), col_scheme, table_scheme])]
    table = Aligner(0, colpath=0)
    try:
        for b, want_col in zip(batches, (1, 1)):
            col = gpu_paths(aligner, b)
            used = {e["column"] for e in aligner.bin_stats() if e["pass"] == 2 and e["pairs"] and e["precision"] == 16}
            assert used == {want_col}, used
            plain = gpu_paths(table, b)
            for x, y in zip(col, plain):
                assert np.array_equal(x, y)
            assert_paths_equal(b, col, np.arange(0, b.n_pairs, 7))
    finally:
        table.close()


def test_box_sweep_family_launches_agree(aligner):
    """One box-sweep launch per lane width (the default) and one launch per
    bin (families = 0) give the same results and paths, and the oracle's
    on a sample; in timing mode the bins of a family launch share its time."""
    from paper_2208_12350_amd.binding import Aligner
    b = W.make_workload("mixed", n_pairs=4000, seed=917)
    fam = gpu_paths(aligner, b)
    per = Aligner(0, families=0)
    timed = Aligner(0, timing=2)
    try:
        plain = gpu_paths(per, b)
        assert not any(e["family_hi"] for e in per.bin_stats() if e["pass"] == 2)
        again = gpu_paths(timed, b)
        st = [e for e in timed.bin_stats() if e["pass"] == 2]
    finally:
        per.close()
        timed.close()
    for x, y, z in zip(fam, plain, again):
        assert np.array_equal(x, y)
        assert np.array_equal(x, z)
    assert any(e["family_hi"] for e in st)
    by_launch = {}
    for e in st:
        by_launch.setdefault(e["launch"], set()).add((e["ms"], e["family_hi"], e["family_lo"]))
    assert all(len(v) == 1 for v in by_launch.values())
    assert_paths_equal(b, fam, np.arange(0, b.n_pairs, 13))


def test_max_query_leaves_unreachable_path_bins_unlaunched():
    """With the caller's bound on query lengths, the path-sweep bins for taller
    boxes, and the int32 bins when no score can leave the packed range, are
    not launched; the paths are those of an unbounded handle and the oracle's.
    A scheme whose best score times the bound exceeds the packed range keeps
    the int32 bins."""
    from paper_2208_12350_amd.binding import Aligner
    b = W.make_workload("dna_small", n_pairs=2000, seed=77)
    longest = int(b.q_len().max())
    rng = np.random.default_rng(6)
    M = np.full((4, 4), -60, np.int8)
    np.fill_diagonal(M, 100)
    hi = W.Scheme(M, 120, 20)
    pairs = []
    for n in (300, 500, 700, 900):
        q = rng.integers(0, 4, size=n).astype(np.uint8)
        r = q.copy()
        r[rng.random(n) < 0.05] = 0
        pairs.append((q, np.concatenate([rng.integers(0, 4, size=20), r]).astype(np.uint8)))
    big = W.from_pairs(pairs, [0] * len(pairs), [hi])
    def launched(al):
        # timing mode: a bin that was not launched reports no time
        return {(e["precision"], e["lanes"], e["rows"]) for e in al.bin_stats() if e["pass"] == 2 and e["ms"] > 0}

    plain = Aligner(0, timing=2)
    try:
        for batch, bound, want_i32 in ((b, longest, False), (big, 900, True)):
            want = gpu_paths(plain, batch)
            every = launched(plain)
            bounded = Aligner(0, max_query=bound, timing=2)
            try:
                got = gpu_paths(bounded, batch)
                some = launched(bounded)
                st = [e for e in bounded.bin_stats() if e["pass"] == 2]
            finally:
                bounded.close()
            for x, y in zip(got, want):
                assert np.array_equal(x, y)
            assert_paths_equal(batch, got, np.arange(0, batch.n_pairs, 5))
            # fewer launches, among them every bin that took pairs
            assert some < every, (sorted(some), sorted(every))
            assert all((e["precision"], e["lanes"], e["rows"]) in some for e in st if e["pairs"])
            assert max(e["lanes"] * e["rows"] for e in st if (e["precision"], e["lanes"], e["rows"]) in some) \
                < max(e["lanes"] * e["rows"] for e in st)
            assert any(key[0] == 32 for key in some) == want_i32
    finally:
        plain.close()
