"""Pins for the oracle's alignment paths (the traceback of Fig. 2(c)).

* hand-derived paths in golden/cigar_cases.txt, including gap placements
  that the tie rule decides;
* exhaustive enumeration of every alignment on tiny inputs (brute.py): the
  path must be the optimal alignment with the reported start and end whose
  traceback choices are smallest, for asymmetric matrices and every gap
  setting, with enough ties that the rule is exercised;
* invariants on workload samples, checked by a scorer that walks the runs
  (not the oracle's matrices): the runs consume exactly the reported
  query and reference intervals, begin and end with a substitution column,
  mark '=' exactly where the residue codes are equal, and score S.
"""
import os

import numpy as np
import pytest

from brute import brute_cigar
from oracle import oracle as O
from paper_2208_12350_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cigar_cases.txt")
GAPS = [(6, 1), (11, 1), (1, 1), (3, 1), (2, 2), (3, 0), (5, 2)]


def _scheme(M, o, e):
    return W.Scheme(np.ascontiguousarray(np.asarray(M, dtype=np.int8)), o, e)


def _fig2():
    M = np.full((4, 4), -2, np.int8)
    np.fill_diagonal(M, 2)
    return _scheme(M, 1, 1)


def test_golden_cigar_cases():
    schemes = {"fig2": _fig2(), "dna": W.dna_scheme()}
    n = 0
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, q, r, want = line.split()
            _, runs = O.cigar_pair(W.encode(q, "ACGT"), W.encode(r, "ACGT"), schemes[name])
            got = O.cigar_string(runs) or "*"
            assert got == want, (line, got)
            n += 1
    assert n >= 10


def _random_matrix(rng, A):
    M = rng.integers(-4, 4, size=(A, A))
    np.fill_diagonal(M, rng.integers(1, 6, size=A))
    return M.astype(np.int8)


@pytest.mark.parametrize("seed", range(3))
def test_cigar_matches_brute_force(seed):
    rng = np.random.default_rng(2000 + seed)
    n_cases = 300
    tied = 0
    for k in range(n_cases):
        A = (2, 3, 4)[k % 3]
        M = _random_matrix(rng, A)
        o, e = GAPS[k % len(GAPS)]
        if k % 2:
            a = rng.integers(0, A, size=int(rng.integers(0, 6)))
            b = rng.integers(0, A, size=int(rng.integers(0, 6)))
        else:
            # flank + run + flank against the same with the run one longer
            # (or shorter), under scores where a gap pays: the gap can sit
            # anywhere in the run, and a mismatch can tie with two gaps
            A = 3
            M = np.full((A, A), -int(rng.integers(2, 5)), np.int8)
            np.fill_diagonal(M, int(rng.integers(4, 6)))
            o, e = ((2, 1), (3, 1), (2, 0), (2, 2), (1, 1))[(k // 2) % 5]
            x = rng.integers(0, A, size=2)
            y = rng.integers(0, A, size=int(rng.integers(1, 3)))
            c, run = int(rng.integers(0, A)), int(rng.integers(1, 3))
            a = np.concatenate([x, [c] * run, y])
            if k % 6 == 4:
                # a substituted run instead: with cheap gaps, a query gap next
                # to a reference gap ties with the reverse order
                d = (c + 1 + int(rng.integers(0, A - 1))) % A
                b = np.concatenate([x, [d] * int(rng.integers(1, 3)), y])
                o, e = ((1, 1), (1, 0))[(k // 6) % 2]
            else:
                b = np.concatenate([x, [c] * (run + 1 if k % 4 == 0 else run - 1), y])
            if k % 8 == 2:
                a, b = b, a
        want_res, want_runs, n_opt = brute_cigar(a, b, M, o, e)
        got_res, got_runs = O.cigar_pair(a, b, _scheme(M, o, e))
        assert got_res == want_res
        assert got_runs.tolist() == want_runs, (a.tolist(), b.tolist(), M.tolist(), o, e,
                                                O.cigar_string(got_runs), O.cigar_string(want_runs))
        tied += int(n_opt > 1)
    # several optimal paths between the same start and end must occur, or
    # the tie rule is not being tested
    assert tied > n_cases // 20, tied


def rescore(runs, q, r, res, M, o, e):
    """Walk the runs over q[q_start..] and r[r_start..]: returns the score
    and the last consumed query and reference positions; checks '=' / 'X'."""
    _, qs, _, rs, _ = res
    i, j, s = qs, rs, 0
    for x in runs:
        n, op = int(x) >> 4, int(x) & 15
        assert n >= 1
        if op in (7, 8):
            for _ in range(n):
                assert (q[i] == r[j]) == (op == 7)
                s += int(M[q[i], r[j]])
                i += 1
                j += 1
        elif op == 1:
            s -= o + (n - 1) * e
            i += n
        elif op == 2:
            s -= o + (n - 1) * e
            j += n
        else:
            raise AssertionError("unknown op %d" % op)
    return s, i - 1, j - 1


def check_runs(runs, q, r, res, scheme):
    sc, qs, qe, rs, re = res
    if sc == 0:
        assert len(runs) == 0
        return
    assert len(runs) >= 1
    assert int(runs[0]) & 15 in (7, 8) and int(runs[-1]) & 15 in (7, 8)
    ops = [int(x) & 15 for x in runs]
    assert all(x != y for x, y in zip(ops, ops[1:])), "adjacent runs of one op"
    s, ie, je = rescore(runs, q, r, res, scheme.matrix, scheme.gap_open, scheme.gap_extend)
    assert (s, ie, je) == (sc, qe, re)


@pytest.mark.parametrize("name", ["dna_small", "protein", "mixed"])
def test_cigar_invariants_on_workload_samples(name):
    b = W.make_workload(name, n_pairs=60)
    res, runs, off, nr = O.cigar_batch(b)
    for i in range(b.n_pairs):
        q, r, s = b.pair(i)
        rr = tuple(int(x) for x in res[i])
        check_runs(runs[off[i]:off[i] + nr[i]], q, r, rr, s)
        # the pairwise entry point agrees with the batch one
        if i < 10:
            res1, runs1 = O.cigar_pair(q, r, s)
            assert res1 == rr and runs1.tolist() == runs[off[i]:off[i] + nr[i]].tolist()


def test_cigar_subset_and_given_results():
    b = W.make_workload("dna_small", n_pairs=40)
    res, runs, off, nr = O.cigar_batch(b)
    idx = [5, 2, 2, 39]
    res2, runs2, off2, nr2 = O.cigar_batch(b, index=idx, threads=2, results=res[idx])
    for k, i in enumerate(idx):
        assert tuple(res2[k]) == tuple(res[i])
        assert runs2[off2[k]:off2[k] + nr2[k]].tolist() == runs[off[i]:off[i] + nr[i]].tolist()


# Inputs on which the walk back meets a gap cell where opening and extending
# the gap both continue an optimal path (found by a seeded search over random
# pairs; the expected paths come from brute force).  The first six meet it in
# a query gap (F), the others in a reference gap (E).  Format: query,
# reference, match score, mismatch score, alphabet, o, e.
OPEN_OR_EXTEND = [
    ([0, 2, 1, 1, 2, 0], [0, 1, 0], 5, -3, 3, 2, 1),
    ([2, 1, 1, 0, 0, 1, 1, 2], [2, 0, 2, 2], 2, -3, 3, 1, 0),
    ([1, 0, 2, 2, 2, 0, 1, 2], [1, 2, 1, 2], 5, -1, 3, 1, 0),
    ([2, 1, 1, 0, 2, 0], [2, 0, 1, 2], 3, -1, 3, 1, 0),
    ([2, 1, 0, 2, 2, 1, 1, 0], [1, 2, 0], 4, -3, 3, 1, 0),
    ([0, 1, 1, 2, 0, 0, 2, 1], [0, 1, 0, 1], 2, -2, 3, 1, 0),
    ([2, 0, 2, 0], [0, 1, 2, 1, 2, 1, 0], 2, -2, 3, 1, 0),
    ([1, 2, 1, 2], [1, 0, 2, 2, 1, 1, 2], 2, -2, 3, 1, 0),
    ([2, 0, 1, 2], [2, 0, 2, 1, 1, 0, 0, 2], 2, -3, 3, 1, 0),
    ([1, 0, 1, 1], [1, 2, 0, 2, 0, 2, 1, 0], 5, -3, 3, 1, 0),
    ([0, 0, 2, 1], [0, 1, 2, 2, 0, 1, 2, 0], 5, -2, 3, 2, 1),
    ([2, 0, 2, 2], [2, 1, 1, 0, 0, 1, 2, 2], 4, -2, 3, 1, 0),
]


@pytest.mark.parametrize("case", OPEN_OR_EXTEND)
def test_cigar_open_or_extend_ties(case):
    a, b, match, mis, A, o, e = case
    M = np.full((A, A), mis, np.int8)
    np.fill_diagonal(M, match)
    want_res, want_runs, n_opt = brute_cigar(a, b, M, o, e)
    assert n_opt > 1
    got_res, got_runs = O.cigar_pair(np.array(a), np.array(b), _scheme(M, o, e))
    assert got_res == want_res
    assert got_runs.tolist() == want_runs, (O.cigar_string(got_runs), O.cigar_string(want_runs))
