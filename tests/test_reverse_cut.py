"""The reverse sweep only covers the part of the reversed prefixes that can
hold a cell of the best score S (the extent rule of the library's reverse
pass, restated here): every cell of score S closes an alignment that spans
exactly p query and q reference residues, which needs |p - q| gap residues,
so q - p (and p - q) is at most the number of gap residues whose least cost
fits in max_score * p - S.  This checks, against a brute-force reverse DP
from the oracle's results, that no cell of score S lies outside the cut,
over gap settings with o > e, o = e, o < e and e = 0."""
import numpy as np

from oracle import oracle as O
from paper_2208_12350_amd import workloads as W

NO_BOUND = 60000


def gap_room(slack, o, e):
    if slack < o:
        return 0
    k = slack // o if o < e else (NO_BOUND if e == 0 else 1 + (slack - o) // e)
    return min(k, NO_BOUND)


def cut(S, mx, o, e, n, m):
    m = min(m, n + gap_room(mx * n - S, o, e))
    n = min(n, m + gap_room(mx * m - S, o, e))
    return n, m


def reverse_scores(a, b, M, o, e):
    n, m = len(a), len(b)
    H = np.zeros((n + 1, m + 1), np.int64)
    E = np.full((n + 1, m + 1), -o, np.int64)
    F = E.copy()
    for i in range(1, n + 1):
        for j in range(1, m + 1):
            E[i, j] = max(E[i, j - 1] - e, H[i, j - 1] - o)
            F[i, j] = max(F[i - 1, j] - e, H[i - 1, j] - o)
            H[i, j] = max(0, H[i - 1, j - 1] + M[a[i - 1], b[j - 1]], E[i, j], F[i, j])
    return H


def test_every_best_cell_of_the_reverse_sweep_is_inside_the_cut():
    rng = np.random.default_rng(1)
    checked = cut_some = 0
    for _ in range(800):
        o, e = int(rng.integers(1, 8)), int(rng.integers(0, 4))
        M = rng.integers(-4, 2, size=(4, 4))
        np.fill_diagonal(M, rng.integers(1, 6, size=4))
        n, m = int(rng.integers(1, 25)), int(rng.integers(1, 40))
        a, b = rng.integers(0, 4, size=n), rng.integers(0, 4, size=m)
        if rng.random() < 0.5:   # a similar segment, so that long alignments occur
            k = min(n, m)
            s0 = int(rng.integers(0, m - k + 1))
            b[s0:s0 + k] = a[:k]
            b[rng.random(m) < 0.15] = rng.integers(0, 4)
        sc = W.Scheme(np.ascontiguousarray(M.astype(np.int8)), o, e)
        S, qs, qe, rs, re_ = O.align_pair(a.astype(np.uint8), b.astype(np.uint8), sc)
        if S <= 0:
            continue
        H = reverse_scores(a[:qe + 1][::-1], b[:re_ + 1][::-1], M, o, e)
        nc, mc = cut(S, int(M.max()), o, e, qe + 1, re_ + 1)
        ps, qs_ = np.nonzero(H == S)
        assert ps.max() <= nc and qs_.max() <= mc, (o, e, S, (qe + 1, re_ + 1), (nc, mc))
        # the first S cell in row-major order is the oracle's start
        k = np.lexsort((qs_, ps))[0]
        assert (qe - ps[k] + 1, re_ - qs_[k] + 1) == (qs, rs)
        checked += 1
        cut_some += (nc, mc) != (qe + 1, re_ + 1)
    assert checked > 500 and cut_some > 50
