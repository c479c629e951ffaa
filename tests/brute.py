"""Brute-force local alignment by enumerating every alignment.

Independent of both the oracle and the GPU path: it never fills a dynamic
programming matrix.  A local alignment of a (query) and b (reference) is a
string of columns -- M (a_i over b_j), I (a_i over a gap) and D (a gap over
b_j) -- covering a[i0..i1] and b[j0..j1].  Its score is the sum of the
substitution scores of its M columns minus, for every maximal run of k
consecutive I columns or k consecutive D columns, the affine cost
o + (k-1)*e (Section II-B-1, generalised from the linear gap of the worked
example to an affine one).

An optimal alignment never begins or ends with a gap column when o >= 1
(dropping it raises the score), so only alignments that begin and end with
an M column are enumerated.  Among all alignments of maximal score S the
reported end is the row-major-first one (smallest i1, then smallest j1) and
the reported start, among optimal alignments with that end, the latest one
(largest i0, then largest j0).  S == 0 gives all coordinates -1.
"""
from __future__ import annotations

import numpy as np


def brute_align(a, b, M, o, e):
    """Return (score, q_start, q_end, r_start, r_end) by exhaustive search."""
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    n, m = len(a), len(b)
    M = np.asarray(M)
    best = 0
    ends = {}  # (i1, j1) -> set of starts achieving the running best
    results = []  # (score, i0, j0, i1, j1)
    for i0 in range(n):
        for j0 in range(m):
            # explicit stack of (i, j, last_column, score); (i, j) = next unconsumed residues
            stack = [(i0 + 1, j0 + 1, "M", int(M[a[i0], b[j0]]))]
            while stack:
                i, j, last, s = stack.pop()
                if last == "M":
                    results.append((s, i0, j0, i - 1, j - 1))
                if i < n and j < m:
                    stack.append((i + 1, j + 1, "M", s + int(M[a[i], b[j]])))
                if i < n:
                    stack.append((i + 1, j, "I", s - (e if last == "I" else o)))
                if j < m:
                    stack.append((i, j + 1, "D", s - (e if last == "D" else o)))
    if not results:
        return (0, -1, -1, -1, -1)
    best = max(r[0] for r in results)
    if best <= 0:
        return (0, -1, -1, -1, -1)
    opt = [r for r in results if r[0] == best]
    i1, j1 = min((r[3], r[4]) for r in opt)
    i0, j0 = max((r[1], r[2]) for r in opt if (r[3], r[4]) == (i1, j1))
    return (best, i0, i1, j0, j1)


def brute_h_matrix(a, b, M, o, e):
    """The (n+1) x (m+1) local-alignment score matrix by enumeration: entry
    [i][j] is the best score of any alignment that consumes a[..i-1] and
    b[..j-1] as its last query and reference residues (its last column may
    be a substitution or either kind of gap), or 0 if none is positive.
    Alignments are enumerated from every first substitution column; one
    that begins with a gap column never scores more than the same alignment
    without it."""
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    n, m = len(a), len(b)
    M = np.asarray(M)
    H = np.zeros((n + 1, m + 1), np.int64)
    for i0 in range(n):
        for j0 in range(m):
            stack = [(i0 + 1, j0 + 1, "M", int(M[a[i0], b[j0]]))]
            while stack:
                i, j, last, s = stack.pop()
                if s > H[i, j]:
                    H[i, j] = s
                if i < n and j < m:
                    stack.append((i + 1, j + 1, "M", s + int(M[a[i], b[j]])))
                if i < n:
                    stack.append((i + 1, j, "I", s - (e if last == "I" else o)))
                if j < m:
                    stack.append((i, j + 1, "D", s - (e if last == "D" else o)))
    return H


def _all_alignments(a, b, M, o, e):
    """Every local alignment that begins and ends with an M column, as
    (score, i0, j0, i1, j1, columns)."""
    n, m = len(a), len(b)
    out = []
    for i0 in range(n):
        for j0 in range(m):
            stack = [(i0 + 1, j0 + 1, ("M",), int(M[a[i0], b[j0]]))]
            while stack:
                i, j, cols, s = stack.pop()
                last = cols[-1]
                if last == "M":
                    out.append((s, i0, j0, i - 1, j - 1, cols))
                if i < n and j < m:
                    stack.append((i + 1, j + 1, cols + ("M",), s + int(M[a[i], b[j]])))
                if i < n:
                    stack.append((i + 1, j, cols + ("I",), s - (e if last == "I" else o)))
                if j < m:
                    stack.append((i, j + 1, cols + ("D",), s - (e if last == "D" else o)))
    return out


def _choice_key(cols, o, e):
    """The choices a traceback makes to spell `cols`, read from the last
    column back: 0 / 1 / 2 for a substitution / query-gap / reference-gap
    column entered from the cell state H, and inside a gap run 1 to extend
    it further back, 0 to stop (the run opens here).  When o == e every gap
    column is its own run (opening costs the same as extending)."""
    key = []
    k = len(cols) - 1
    while k >= 0:
        c = cols[k]
        if c == "M":
            key.append(0)
            k -= 1
            continue
        q = k
        while q > 0 and cols[q - 1] == c:
            q -= 1
        run = k - q + 1
        d = 1 if c == "I" else 2
        if o == e:
            key.extend([d, 0] * run)
        else:
            key.extend([d] + [1] * (run - 1) + [0])
        k = q - 1
    return key


def brute_cigar(a, b, M, o, e):
    """(result, runs) by exhaustive search: the result of brute_align, and
    among the optimal alignments with its start and end the one whose
    traceback choices (``_choice_key``) are smallest.  Runs are
    (length << 4) | op with the SAM codes 7 '=', 8 'X', 1 'I', 2 'D'.  Also
    returns how many optimal alignments shared that start and end."""
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    M = np.asarray(M)
    alns = _all_alignments(a, b, M, o, e)
    best = max((x[0] for x in alns), default=0)
    if best <= 0:
        return (0, -1, -1, -1, -1), [], 0
    opt = [x for x in alns if x[0] == best]
    i1, j1 = min((x[3], x[4]) for x in opt)
    i0, j0 = max((x[1], x[2]) for x in opt if (x[3], x[4]) == (i1, j1))
    cand = [x[5] for x in opt if (x[1], x[2], x[3], x[4]) == (i0, j0, i1, j1)]
    cols = min(cand, key=lambda c: _choice_key(c, o, e))
    ops = []
    i, j = i0, j0
    for c in cols:
        if c == "M":
            ops.append(7 if a[i] == b[j] else 8)
            i += 1
            j += 1
        elif c == "I":
            ops.append(1)
            i += 1
        else:
            ops.append(2)
            j += 1
    runs = []
    for op in ops:
        if runs and (runs[-1] & 15) == op:
            runs[-1] += 16
        else:
            runs.append(16 | op)
    return (best, i0, i1, j0, j1), runs, len(cand)
