"""Pins for the CPU oracle: it is checked against things other than itself.

* exhaustive enumeration of every local alignment on tiny inputs (brute.py),
  with asymmetric matrices so a transposed matrix index fails, several gap
  settings so a wrong open/extend term fails, and enough ties that the
  row-major-first end and latest-start rules are exercised;
* the hand-derived cases in golden/hand_cases.txt (the Fig. 2 worked example
  parameters of Section II-B-1 among them);
* closed forms and special cases: self-alignment, exact embedding, o == e is
  the textbook linear-gap recurrence, prohibitive gaps reduce to the best
  diagonal run (Kadane's maximum subarray);
* invariants: score >= 0, the -1 sentinel, coordinate ranges, re-scoring the
  reported substrings by global alignment gives S, query/reference swap under
  a symmetric matrix, scaling of every score by k, monotonicity in the
  reference.
"""
import os

import numpy as np
import pytest

from brute import brute_align, brute_h_matrix
from oracle import oracle as O
from paper_2208_12350_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_cases.txt")


def _scheme(M, o, e):
    return W.Scheme(np.ascontiguousarray(np.asarray(M, dtype=np.int8)), o, e)


def _fig2():
    M = np.full((4, 4), -2, np.int8)
    np.fill_diagonal(M, 2)
    return _scheme(M, 1, 1)


def test_golden_hand_cases():
    schemes = {"fig2": _fig2(), "dna": W.dna_scheme()}
    n = 0
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, q, r, *exp = line.split()
            got = O.align_pair(W.encode(q, "ACGT"), W.encode(r, "ACGT"), schemes[name])
            assert got == tuple(int(x) for x in exp), (line, got)
            n += 1
    assert n >= 8


GAPS = [(6, 1), (11, 1), (1, 1), (3, 1), (2, 2), (3, 0), (5, 2)]


def _random_matrix(rng, A, symmetric):
    M = rng.integers(-4, 4, size=(A, A))
    if symmetric:
        M = np.triu(M, 1)
        M = M + M.T
    np.fill_diagonal(M, rng.integers(1, 6, size=A))
    return M.astype(np.int8)


@pytest.mark.parametrize("seed", range(4))
def test_oracle_matches_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    n_cases = 500
    ties_end = 0
    for k in range(n_cases):
        A = (2, 4, 6)[k % 3]
        M = _random_matrix(rng, A, symmetric=(k % 4 == 0))
        o, e = GAPS[k % len(GAPS)]
        a = rng.integers(0, A, size=int(rng.integers(0, 6)))
        b = rng.integers(0, A, size=int(rng.integers(0, 7)))
        want = brute_align(a, b, M, o, e)
        got = O.align_pair(a, b, _scheme(M, o, e))
        assert got == want, (a.tolist(), b.tolist(), M.tolist(), o, e, got, want)
        if want[0] > 0:
            H = O.score_matrix(a, b, _scheme(M, o, e))
            ties_end += int(np.sum(H == want[0]) > 1)
    # ties must actually occur, or the tie-break rules are not being tested
    assert ties_end > n_cases // 20


@pytest.mark.parametrize("seed", range(2))
def test_score_matrix_matches_brute_force(seed):
    """The full H matrix the oracle returns equals the enumerated one cell by
    cell; its maximum is the score of align_pair and its row-major-first
    maximum is the reported end."""
    rng = np.random.default_rng(3000 + seed)
    for k in range(300):
        A = (2, 4, 6)[k % 3]
        M = _random_matrix(rng, A, symmetric=(k % 4 == 0))
        o, e = GAPS[k % len(GAPS)]
        a = rng.integers(0, A, size=int(rng.integers(0, 6)))
        b = rng.integers(0, A, size=int(rng.integers(0, 6)))
        H = O.score_matrix(a, b, _scheme(M, o, e))
        want = brute_h_matrix(a, b, M, o, e)
        assert H.shape == (a.size + 1, b.size + 1)
        assert np.array_equal(H, want), (a.tolist(), b.tolist(), M.tolist(), o, e, H.tolist(), want.tolist())
        S, _, qe, _, re = brute_align(a, b, M, o, e)
        assert int(H.max()) == S
        if S > 0:
            i, j = np.argwhere(H == S)[0]          # row-major first
            assert (int(i) - 1, int(j) - 1) == (qe, re)


def test_batch_equals_pairwise():
    b = W.make_workload("dna_small", n_pairs=50)
    out = O.align_batch(b, threads=3)
    for i in range(b.n_pairs):
        q, r, s = b.pair(i)
        assert tuple(int(x) for x in out[i]) == O.align_pair(q, r, s)
    sub = O.align_batch(b, index=[7, 3, 3, 0], threads=2)
    assert np.array_equal(sub, out[[7, 3, 3, 0]])


def test_empty_and_invalid():
    s = W.dna_scheme()
    assert O.align_pair(np.zeros(0, np.uint8), W.encode("ACGT", "ACGT"), s) == (0, -1, -1, -1, -1)
    assert O.align_pair(W.encode("ACGT", "ACGT"), np.zeros(0, np.uint8), s) == (0, -1, -1, -1, -1)
    with pytest.raises(ValueError):
        O.align_pair(np.array([0, 4], np.uint8), W.encode("ACGT", "ACGT"), s)


def test_self_alignment_closed_form():
    """If M[x][x] > 0 and every off-diagonal entry is below both diagonal
    entries, aligning a sequence with itself scores the sum of its diagonal
    scores, over the whole sequence."""
    rng = np.random.default_rng(5)
    for scheme in (W.dna_scheme(), W.protein_scheme(11)):
        A = scheme.alphabet
        for _ in range(40):
            a = rng.integers(0, A, size=int(rng.integers(1, 300))).astype(np.uint8)
            S = int(np.sum(scheme.matrix[a, a].astype(np.int64)))
            assert O.align_pair(a, a, scheme) == (S, 0, a.size - 1, 0, a.size - 1)


def test_exact_embedding_closed_form():
    rng = np.random.default_rng(6)
    s = W.dna_scheme()
    for _ in range(40):
        q = rng.integers(0, 4, size=int(rng.integers(40, 120))).astype(np.uint8)
        left = rng.integers(0, 4, size=int(rng.integers(0, 80))).astype(np.uint8)
        right = rng.integers(0, 4, size=int(rng.integers(0, 80))).astype(np.uint8)
        r = np.concatenate([left, q, right])
        got = O.align_pair(q, r, s)
        assert got == (3 * q.size, 0, q.size - 1, left.size, left.size + q.size - 1)


def _linear_sw(a, b, M, g):
    """Textbook linear-gap Smith-Waterman: H = max(0, diag + s, up - g, left - g)."""
    n, m = len(a), len(b)
    H = np.zeros((n + 1, m + 1), np.int64)
    for i in range(1, n + 1):
        for j in range(1, m + 1):
            H[i, j] = max(0, H[i - 1, j - 1] + int(M[a[i - 1], b[j - 1]]), H[i - 1, j] - g, H[i, j - 1] - g)
    S = int(H.max())
    if S == 0:
        return 0, -1, -1
    i, j = np.argwhere(H == S)[0]  # argwhere is row-major
    return S, int(i) - 1, int(j) - 1


def test_equal_open_and_extend_is_linear_gap_sw():
    rng = np.random.default_rng(7)
    for k in range(200):
        A = 4
        M = _random_matrix(rng, A, symmetric=False)
        g = int(rng.integers(1, 4))
        a = rng.integers(0, A, size=int(rng.integers(1, 25)))
        b = rng.integers(0, A, size=int(rng.integers(1, 25)))
        S, qe, re = _linear_sw(a, b, M, g)
        got = O.align_pair(a, b, _scheme(M, g, g))
        assert (got[0], got[2], got[4]) == (S, qe, re)


def test_prohibitive_gaps_is_best_diagonal_run():
    """With gap costs above any achievable score no gap is ever taken, and the
    score is the best maximum-subarray sum over the diagonals of the score
    grid; the end is the row-major-first cell ending such a run."""
    rng = np.random.default_rng(8)
    for _ in range(200):
        A = 4
        M = _random_matrix(rng, A, symmetric=False)
        a = rng.integers(0, A, size=int(rng.integers(1, 30)))
        b = rng.integers(0, A, size=int(rng.integers(1, 30)))
        big = 10 * 6 * (len(a) + len(b))
        n, m = len(a), len(b)
        best = 0
        best_end = (-1, -1)
        runs = {}
        for i in range(n):
            for j in range(m):
                s = int(M[a[i], b[j]])
                prev = runs.get((i - 1, j - 1), 0)
                cur = max(s, prev + s) if prev > 0 else s
                runs[(i, j)] = max(cur, 0)
                if cur > best:
                    best, best_end = cur, (i, j)
        got = O.align_pair(a, b, _scheme(M, big, big))
        assert got[0] == best
        if best > 0:
            assert (got[2], got[4]) == best_end


def _global_gotoh(a, b, M, o, e):
    """Best global alignment score of a against b (all residues aligned)."""
    n, m = len(a), len(b)
    NEG = -10 ** 12
    H = np.full((n + 1, m + 1), NEG, np.int64)
    E = np.full((n + 1, m + 1), NEG, np.int64)
    F = np.full((n + 1, m + 1), NEG, np.int64)
    H[0, 0] = 0
    for j in range(1, m + 1):
        E[0, j] = -(o + (j - 1) * e)
        H[0, j] = E[0, j]
    for i in range(1, n + 1):
        F[i, 0] = -(o + (i - 1) * e)
        H[i, 0] = F[i, 0]
        for j in range(1, m + 1):
            E[i, j] = max(E[i, j - 1] - e, H[i, j - 1] - o)
            F[i, j] = max(F[i - 1, j] - e, H[i - 1, j] - o)
            H[i, j] = max(H[i - 1, j - 1] + int(M[a[i - 1], b[j - 1]]), E[i, j], F[i, j])
    return int(H[n, m])


@pytest.mark.parametrize("name", ["dna_small", "protein"])
def test_invariants_on_workload_samples(name):
    b = W.make_workload(name, n_pairs=40)
    out = O.align_batch(b)
    for i in range(b.n_pairs):
        q, r, s = b.pair(i)
        sc, qs, qe, rs, re = (int(x) for x in out[i])
        assert sc >= 0
        if sc == 0:
            assert (qs, qe, rs, re) == (-1, -1, -1, -1)
            continue
        assert 0 <= qs <= qe < q.size and 0 <= rs <= re < r.size
        if (qe - qs + 1) * (re - rs + 1) <= 60_000:
            assert _global_gotoh(q[qs:qe + 1], r[rs:re + 1], s.matrix, s.gap_open, s.gap_extend) == sc
        # a local alignment of the reported substrings alone reaches the same score
        assert O.align_pair(q[qs:qe + 1], r[rs:re + 1], s)[0] == sc


def test_swap_symmetry_and_scaling():
    rng = np.random.default_rng(9)
    for k in range(100):
        A = 4 if k % 2 else 20
        M = _random_matrix(rng, A, symmetric=True)
        o, e = GAPS[k % len(GAPS)]
        if o < e:
            continue
        a = rng.integers(0, A, size=int(rng.integers(1, 60)))
        b = rng.integers(0, A, size=int(rng.integers(1, 60)))
        x = O.align_pair(a, b, _scheme(M, o, e))
        y = O.align_pair(b, a, _scheme(M, o, e))
        assert x[0] == y[0]
        kk = int(rng.integers(2, 6))
        z = O.align_pair(a, b, _scheme(M.astype(np.int64) * kk, o * kk, e * kk))
        assert z == (x[0] * kk,) + x[1:]


def test_monotone_in_reference():
    rng = np.random.default_rng(10)
    s = W.dna_scheme()
    for _ in range(100):
        a = rng.integers(0, 4, size=int(rng.integers(1, 40)))
        b = rng.integers(0, 4, size=int(rng.integers(1, 40)))
        ext = np.concatenate([b, rng.integers(0, 4, size=int(rng.integers(1, 10)))])
        assert O.align_pair(a, ext, s)[0] >= O.align_pair(a, b, s)[0]
