"""Database search (sw_search, one query against many references) against
the oracle: every pair of a small set, a sample of the full-size DNA search,
properties over all pairs, and agreement with sw_align_batch on the same
pairs given one by one."""
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


def run_search(aligner, s, query=None):
    import torch
    dev = "cuda:0"
    q = torch.from_numpy(np.ascontiguousarray(s.query if query is None else query)).to(dev)
    r = torch.from_numpy(s.refs).to(dev)
    ro = torch.from_numpy(s.r_off).to(dev)
    return aligner.search(q, r, ro, s.scheme).cpu().numpy().astype(np.int64)


def oracle_rows(s, idx):
    o = O.align_batch(s.as_batch(idx))
    return np.stack([o[f] for f in FIELDS], axis=1).astype(np.int64)


def test_protein_search_every_pair(aligner):
    s = W.make_search("search_protein", n_refs=3000)
    got = run_search(aligner, s)
    assert np.array_equal(got, oracle_rows(s, np.arange(s.n_refs)))


def test_full_size_dna_search_sampled(aligner):
    s = W.make_search("search_dna")
    got = run_search(aligner, s)
    idx = np.sort(np.random.default_rng(4).choice(s.n_refs, size=300, replace=False))
    idx = np.union1d(idx, np.flatnonzero(s.homolog)[:50])
    assert np.array_equal(got[idx], oracle_rows(s, idx))
    # every homologue outscores every unrelated reference
    assert got[s.homolog, 0].min() > got[~s.homolog, 0].max()
    # coordinates lie inside the query and each reference
    pos = got[:, 0] > 0
    rl = np.diff(s.r_off)
    assert np.all((got[pos, 1] >= 0) & (got[pos, 1] <= got[pos, 2]) & (got[pos, 2] < s.query.size))
    assert np.all((got[pos, 3] >= 0) & (got[pos, 3] <= got[pos, 4]) & (got[pos, 4] < rl[pos]))


def test_search_equals_batch_and_changes_query_length(aligner):
    from paper_2208_12350_amd.binding import DeviceBatch
    s = W.make_search("search_protein", n_refs=5000)
    got = run_search(aligner, s)
    b = s.as_batch()
    want = aligner.align(DeviceBatch.from_host(b)).cpu().numpy().astype(np.int64)
    assert np.array_equal(got, want)
    # a shorter query, then the original again (the stored spans are refilled)
    short = s.query[:123].copy()
    got2 = run_search(aligner, s, short)
    s2 = W.SearchSet(short, s.refs, s.r_off, s.scheme)
    idx = np.arange(0, s.n_refs, 7)
    assert np.array_equal(got2[idx], oracle_rows(s2, idx))
    assert np.array_equal(run_search(aligner, s), got)


def test_empty_and_too_long_queries(aligner):
    from paper_2208_12350_amd.binding import SwError
    s = W.make_search("search_dna", n_refs=100)
    got = run_search(aligner, s, np.zeros(0, np.uint8))
    assert np.all(got == [0, -1, -1, -1, -1])
    with pytest.raises(SwError):
        run_search(aligner, s, np.zeros(2049, np.uint8))


@pytest.mark.parametrize("n_q", [1, 7, 16, 100, 257, 400, 513, 1024, 1500, 2048])
def test_query_profile_equals_pair_table_and_oracle(n_q):
    """The forward pass of a protein search reads its scores from the query
    profile (every query length routes to some shape, 16 to 64 lanes; above
    512 rows the routing may pick cooperative groups, which keep the pair
    table): the same bits as the pair-table path, and the oracle's on a
    sample of pairs that includes the homologues."""
    import torch
    from paper_2208_12350_amd.binding import Aligner
    s = W.make_search("search_protein", n_refs=2500, seed=600 + n_q)
    rng = np.random.default_rng(n_q)
    query = rng.integers(0, 20, size=n_q).astype(np.uint8)
    query[:min(n_q, 400)] = s.query[:min(n_q, 400)]
    dev = "cuda:0"
    q = torch.from_numpy(query).to(dev)
    r = torch.from_numpy(s.refs).to(dev)
    ro = torch.from_numpy(s.r_off).to(dev)
    outs = []
    for qp in (1, 0):
        al = Aligner(0, qprofile=qp)
        try:
            outs.append(al.search(q, r, ro, s.scheme).cpu().numpy().astype(np.int64))
            if qp == 0:
                assert al.get_option("qprofile_used") == 0
            else:
                used = al.get_option("qprofile_used")
                assert used == 1
                # the forward launches that ran: every one of them on a profile
                # kernel, unless the shape is a cooperative group
                fwd = [e for e in al.bin_stats() if e["pass"] == 0 and e["pairs"] > 0]
                assert all(e["column"] == 3 or e["lanes"] > 64 for e in fwd)
        finally:
            al.close()
    assert np.array_equal(outs[0], outs[1])
    s2 = W.SearchSet(query, s.refs, s.r_off, s.scheme)
    idx = np.union1d(np.arange(0, s.n_refs, 9), np.flatnonzero(s.homolog))
    assert np.array_equal(outs[0][idx], oracle_rows(s2, idx))


def test_dna_search_keeps_column_words():
    """A DNA search takes the column-word path (no pair table, no profile)."""
    import torch
    from paper_2208_12350_amd.binding import Aligner
    s = W.make_search("search_dna", n_refs=2000)
    al = Aligner(0)
    try:
        dev = "cuda:0"
        got = al.search(torch.from_numpy(s.query).to(dev), torch.from_numpy(s.refs).to(dev),
                        torch.from_numpy(s.r_off).to(dev), s.scheme).cpu().numpy().astype(np.int64)
        assert al.get_option("qprofile_used") == 0
    finally:
        al.close()
    idx = np.arange(0, s.n_refs, 5)
    assert np.array_equal(got[idx], oracle_rows(s, idx))


@pytest.mark.parametrize("case", ["high_scores", "long_refs", "forced_int32"])
def test_search_pairs_on_int32_bins(case):
    """A search's forward pass launches only its query length's bins, the
    packed int16 one and the int32 one: pairs that need int32 (scores past
    the packed range, references above 32,000 residues, or the precision
    forced to 32 bits) come out as the oracle's, next to int16 pairs of the
    same search."""
    import torch
    from paper_2208_12350_amd.binding import Aligner
    rng = np.random.default_rng({"high_scores": 1, "long_refs": 2, "forced_int32": 3}[case])
    n_q = 400
    query = rng.integers(0, 4, size=n_q).astype(np.uint8)
    lens = rng.integers(100, 600, size=120)
    if case == "long_refs":
        lens[[5, 60, 119]] = 33000
    refs = []
    for k, L in enumerate(lens):
        r = rng.integers(0, 4, size=int(L)).astype(np.uint8)
        if k % 3 == 0 and L > n_q:
            at = int(rng.integers(0, L - n_q))
            r[at:at + n_q] = query   # a homologue: the whole query matches
        refs.append(r)
    r_off = np.zeros(len(refs) + 1, np.int64)
    np.cumsum([r.size for r in refs], out=r_off[1:])
    # match 100: 400 matching rows score 40,000, past the packed int16 range
    scheme = W.dna_scheme(match=100, mismatch=-60, gap_open=150, gap_extend=20) if case == "high_scores" \
        else W.dna_scheme()
    s = W.SearchSet(query, np.concatenate(refs), r_off, scheme)
    al = Aligner(0, precision=32) if case == "forced_int32" else Aligner(0)
    try:
        dev = "cuda:0"
        got = al.search(torch.from_numpy(query).to(dev), torch.from_numpy(s.refs).to(dev),
                        torch.from_numpy(r_off).to(dev), scheme).cpu().numpy().astype(np.int64)
        stats = [e for e in al.bin_stats() if e["pass"] == 0 and e["pairs"] > 0]
        assert sum(e["pairs"] for e in stats) == len(refs)
        i32 = sum(e["pairs"] for e in stats if e["precision"] == 32)
        if case == "forced_int32":
            assert i32 == len(refs)
        elif case == "high_scores":
            # packed int16 holds min(n, m) * 100 <= 30,592, i.e. references of at most 305
            assert i32 == int(np.sum(np.minimum(lens, n_q) * 100 > 30592))
        else:
            assert i32 == 3
    finally:
        al.close()
    idx = np.arange(s.n_refs)
    assert np.array_equal(got, oracle_rows(s, idx))
