"""GPU parity of the pair-table sweep (two rows' scores per LDS load), which
the packed int16 kernels use when exactly one scheme of a call takes table
lookups: bit-identical to the byte-table sweep and to the oracle, over the
shapes' odd and even rows per lane, ragged lengths, the largest alphabet the
table holds and the schemes it must refuse."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_12350_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("score", "q_start", "q_end", "r_start", "r_end")


def _oracle_rows(batch):
    o = O.align_batch(batch)
    return np.stack([o[f] for f in FIELDS], axis=1).astype(np.int64)


def _run(batch, **options):
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch
    al = Aligner(0, **options)
    try:
        out = al.align(DeviceBatch.from_host(batch)).cpu().numpy().astype(np.int64)
        used = al.get_option("pairtable_used")
        i32 = al.stats()[2]
    finally:
        al.close()
    return out, used, i32


def _random_pairs(rng, A, n_pairs, qmax, rmax, p_embed=0.5, p_sub=0.25):
    pairs = []
    for _ in range(n_pairs):
        n = int(rng.integers(1, qmax + 1))
        m = int(rng.integers(1, rmax + 1))
        q = rng.integers(0, A, size=n).astype(np.uint8)
        r = rng.integers(0, A, size=m).astype(np.uint8)
        if m >= n and rng.random() < p_embed:
            mut = q.copy()
            flip = rng.random(n) < p_sub
            mut[flip] = rng.integers(0, A, size=int(flip.sum()))
            off = int(rng.integers(0, m - n + 1))
            r[off:off + n] = mut
        pairs.append((q, r))
    return pairs


def test_protein_pair_table_equals_byte_table_and_oracle():
    rng = np.random.default_rng(91)
    sc = W.protein_scheme(17)
    # every query length up to 512 rows, so every 16- and 32-lane shape
    # (odd and even rows per lane) runs
    pairs = _random_pairs(rng, 20, 2500, 512, 700)
    pairs += [(rng.integers(0, 20, size=n).astype(np.uint8), rng.integers(0, 20, size=m).astype(np.uint8))
              for n in (1, 2, 15, 16, 17, 31, 33, 255, 256, 257, 511, 512) for m in (1, 3, 128, 129, 300)]
    b = W.from_pairs(pairs, [0] * len(pairs), [sc])
    got, used, i32 = _run(b)
    assert used == 1 and i32 == 0
    ref, used0, _ = _run(b, pairtable=0)
    assert used0 == 0
    assert np.array_equal(got, ref)
    assert np.array_equal(got, _oracle_rows(b))


def test_mixed_workload_uses_the_pair_table_for_protein():
    b = W.make_workload("mixed", n_pairs=6000, seed=92)
    got, used, _ = _run(b)
    assert used == 1
    assert np.array_equal(got, _oracle_rows(b))


def test_dna_without_column_words_takes_the_pair_table():
    b = W.make_workload("dna_small", seed=93)
    got, used, _ = _run(b, colpath=0)
    assert used == 1
    assert np.array_equal(got, _oracle_rows(b))


def test_largest_alphabet_and_refused_schemes():
    rng = np.random.default_rng(94)
    # 24 residues: the largest table (25^3 entries)
    M = rng.integers(-5, 3, size=(24, 24))
    M = np.triu(M, 1) + np.triu(M, 1).T
    np.fill_diagonal(M, rng.integers(5, 12, size=24))
    big = W.Scheme(np.ascontiguousarray(M.astype(np.int8)), 9, 2, "a24")
    pairs = _random_pairs(rng, 24, 1500, 300, 500)
    b = W.from_pairs(pairs, [0] * len(pairs), [big])
    got, used, _ = _run(b)
    assert used == 1
    assert np.array_equal(got, _oracle_rows(b))
    # 25 residues: no pair table; a mismatch below -o: no pair table; two
    # table-lookup schemes in one call: no pair table -- each still exact
    M25 = rng.integers(-4, 4, size=(25, 25))
    np.fill_diagonal(M25, 6)
    s25 = W.Scheme(np.ascontiguousarray(M25.astype(np.int8)), 11, 1, "a25")
    Mneg = np.full((20, 20), -20, dtype=np.int8)
    np.fill_diagonal(Mneg, 7)
    sneg = W.Scheme(Mneg, 6, 1, "neg")
    for schemes, A in (([s25], 25), ([sneg], 20), ([W.protein_scheme(3), W.protein_scheme(4)], 20)):
        pairs = _random_pairs(rng, A, 800, 200, 400)
        sids = [k % len(schemes) for k in range(len(pairs))]
        b = W.from_pairs(pairs, sids, schemes)
        got, used, _ = _run(b)
        assert used == 0, [s.name for s in schemes]
        assert np.array_equal(got, _oracle_rows(b))


def test_pair_table_reverse_pass_on_full_protein_sample():
    """The protein workload at full size (100,000 pairs), pair table on, in
    the persistent launch: a seeded sample of pairs against the oracle, every
    pair against the byte-table run."""
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch
    import torch
    b = W.make_workload("protein")
    db = DeviceBatch.from_host(b)
    outs = []
    for pt in (1, 0):
        al = Aligner(0, pairtable=pt)
        try:
            outs.append(al.align(db).cpu().numpy().astype(np.int64))
            assert al.get_option("pairtable_used") == pt
        finally:
            al.close()
    assert np.array_equal(outs[0], outs[1])
    idx = np.sort(np.random.default_rng(95).choice(b.n_pairs, 1500, replace=False))
    want = O.align_batch(b, index=idx)
    assert np.array_equal(outs[0][idx], np.stack([want[f] for f in FIELDS], axis=1).astype(np.int64))
