"""Seeded synthetic alignment workloads.

This module only draws inputs: sequences, substitution matrices, gap
penalties and request arrival times.  It holds none of the alignment
arithmetic, so both the CPU oracle and the GPU path may consume what it
produces without sharing any of the method's code.

The paper's own fitness and held-out sets (30,000 and 4.6 million ADEPT DNA
pairs, Section III-C) are not available here; the generators below stand in
for them with the shapes of the five workloads this library is measured on:

  dna_small   1,000 DNA pairs, query U{50..150}, reference U{100..300}
  dna_large   200,000 DNA pairs, query U{100..256}, reference U{200..600}
  protein     100,000 protein pairs, query U{100..500}, reference U{200..1000}
  mixed       1,000,000 pairs, 80% DNA / 20% protein, log-normal query
              lengths with a 5% long tail, reference 1.5-3x the query
  serving     Poisson stream of requests, each 1-5,000 pairs of the mixed draw

Every reference is built by embedding a mutated copy of its query at a random
offset inside random flanking sequence (see ``mutate_embed``).  Residues are
coded 0..A-1; DNA uses A=4 (ACGT), protein A=20.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

BASE_SEED = 220812350

DNA_ALPHABET = "ACGT"
PROTEIN_ALPHABET = "ARNDCQEGHILKMFPSTWYV"


@dataclasses.dataclass
class Scheme:
    """A scoring scheme: an A x A int8 substitution matrix (row = query
    residue, column = reference residue) and affine gap penalties given as
    positive costs: a gap of length k costs ``gap_open + (k-1)*gap_extend``."""

    matrix: np.ndarray  # int8 [A, A], C-contiguous
    gap_open: int
    gap_extend: int
    name: str = ""

    @property
    def alphabet(self) -> int:
        return int(self.matrix.shape[0])


@dataclasses.dataclass
class Batch:
    """A batch of pairs in the flat layout the C ABI takes.

    queries/refs are concatenated residue codes (uint8); q_off/r_off are
    int64 prefix offsets of length n_pairs+1; scheme_id is uint8 [n_pairs]
    indexing ``schemes``.
    """

    queries: np.ndarray
    q_off: np.ndarray
    refs: np.ndarray
    r_off: np.ndarray
    scheme_id: np.ndarray
    schemes: List[Scheme]
    name: str = ""
    seed: int = 0

    @property
    def n_pairs(self) -> int:
        return int(self.q_off.shape[0] - 1)

    def q_len(self) -> np.ndarray:
        return np.diff(self.q_off)

    def r_len(self) -> np.ndarray:
        return np.diff(self.r_off)

    def cells(self) -> int:
        return int(np.sum(self.q_len().astype(np.int64) * self.r_len().astype(np.int64)))

    def pair(self, i: int):
        q = self.queries[self.q_off[i]:self.q_off[i + 1]]
        r = self.refs[self.r_off[i]:self.r_off[i + 1]]
        return q, r, self.schemes[int(self.scheme_id[i])]

    def subset(self, idx: Sequence[int]) -> "Batch":
        """A new batch holding pairs ``idx`` in that order."""
        return from_pairs([self.pair(int(i))[:2] for i in idx],
                          [int(self.scheme_id[int(i)]) for i in idx],
                          self.schemes, name=self.name + "[subset]", seed=self.seed)


def from_pairs(pairs, scheme_ids, schemes, name="", seed=0) -> Batch:
    """Pack a list of (query, ref) residue arrays into a Batch."""
    qs = [np.asarray(p[0], dtype=np.uint8) for p in pairs]
    rs = [np.asarray(p[1], dtype=np.uint8) for p in pairs]
    q_off = np.zeros(len(qs) + 1, dtype=np.int64)
    r_off = np.zeros(len(rs) + 1, dtype=np.int64)
    q_off[1:] = np.cumsum([len(q) for q in qs])
    r_off[1:] = np.cumsum([len(r) for r in rs])
    queries = np.concatenate(qs) if qs and q_off[-1] > 0 else np.zeros(0, np.uint8)
    refs = np.concatenate(rs) if rs and r_off[-1] > 0 else np.zeros(0, np.uint8)
    return Batch(queries.astype(np.uint8), q_off, refs.astype(np.uint8), r_off,
                 np.asarray(scheme_ids, dtype=np.uint8), list(schemes), name, seed)


def encode(s: str, alphabet: str) -> np.ndarray:
    table = {c: i for i, c in enumerate(alphabet)}
    return np.array([table[c] for c in s], dtype=np.uint8)


# --------------------------------------------------------------------------
# Scoring schemes
# --------------------------------------------------------------------------

def dna_scheme(match: int = 3, mismatch: int = -3, gap_open: int = 6,
               gap_extend: int = 1) -> Scheme:
    m = np.full((4, 4), mismatch, dtype=np.int8)
    np.fill_diagonal(m, match)
    return Scheme(np.ascontiguousarray(m), gap_open, gap_extend, "dna")


def protein_scheme(seed: int) -> Scheme:
    """Seeded symmetric 20x20 int8 matrix: diagonal U{4..11}, off-diagonal
    U{-4..3}; gap open 11, extend 1."""
    rng = np.random.default_rng(seed)
    m = rng.integers(-4, 4, size=(20, 20))
    m = np.triu(m, 1)
    m = m + m.T
    np.fill_diagonal(m, rng.integers(4, 12, size=20))
    return Scheme(np.ascontiguousarray(m.astype(np.int8)), 11, 1, "protein")


def protein_frequencies(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed + 7)
    return rng.dirichlet(np.full(20, 2.0))


# --------------------------------------------------------------------------
# Mutated-embedding generator
# --------------------------------------------------------------------------

def _draw(rng, size, pi: Optional[np.ndarray], A: int) -> np.ndarray:
    if size == 0:
        return np.zeros(0, np.uint8)
    if pi is None:
        return rng.integers(0, A, size=size, dtype=np.uint8)
    return rng.choice(A, size=size, p=pi).astype(np.uint8)


def _substitute(rng, orig: np.ndarray, pi: Optional[np.ndarray], A: int) -> np.ndarray:
    """Replace each residue by one drawn from pi renormalised without it."""
    if orig.size == 0:
        return orig
    if pi is None:
        return ((orig.astype(np.int64) + rng.integers(1, A, size=orig.size)) % A).astype(np.uint8)
    out = _draw(rng, orig.size, pi, A)
    bad = out == orig
    while np.any(bad):
        out[bad] = _draw(rng, int(bad.sum()), pi, A)
        bad = out == orig
    return out


def mutate_embed(rng, q_lens: np.ndarray, r_lens: np.ndarray, p_sub: float,
                 p_indel: float, pi: Optional[np.ndarray], A: int, queries: Optional[np.ndarray] = None):
    """Draw queries of the given lengths and references that embed a mutated
    copy of each query.

    For each query position independently: with probability p_indel it
    becomes an indel (half insertions, which add one residue drawn from pi
    before the position, half deletions, which drop it); otherwise with
    probability p_sub it is substituted.  The reference length becomes
    max(L_r, |copy|); the copy sits at an offset drawn uniformly from
    0..L_r-|copy| and the flanks are iid pi.

    Returns (queries, q_off, refs, r_off) for these pairs.  `queries`
    (concatenated, of the given lengths) replaces the drawn queries.
    """
    q_lens = np.asarray(q_lens, dtype=np.int64)
    r_lens = np.asarray(r_lens, dtype=np.int64)
    P = q_lens.size
    q_off = np.zeros(P + 1, np.int64)
    q_off[1:] = np.cumsum(q_lens)
    Q = int(q_off[-1])
    if queries is None:
        queries = _draw(rng, Q, pi, A)
    else:
        queries = np.ascontiguousarray(queries, dtype=np.uint8)
        if queries.size != Q:
            raise ValueError("queries do not match q_lens")

    u_indel = rng.random(Q)
    u_kind = rng.random(Q)
    u_sub = rng.random(Q)
    is_indel = u_indel < p_indel
    is_ins = is_indel & (u_kind < 0.5)
    is_del = is_indel & ~(u_kind < 0.5)
    is_sub = (~is_indel) & (u_sub < p_sub)

    kept = queries.copy()
    kept[is_sub] = _substitute(rng, queries[is_sub], pi, A)
    # emission per position: [inserted residue] + [kept residue], deletions emit nothing
    n_emit = np.where(is_del, 0, 1) + np.where(is_ins, 1, 0)
    ins_res = _draw(rng, int(is_ins.sum()), pi, A)
    ins_full = np.zeros(Q, np.uint8)
    ins_full[is_ins] = ins_res
    # build the emitted stream: for inserted positions two symbols (ins, kept)
    first = np.where(is_ins, ins_full, kept)
    second = kept
    take_first = n_emit >= 1
    take_second = n_emit == 2
    # interleave first/second in position order
    stream_sym = np.empty(2 * Q, np.uint8)
    stream_sym[0::2] = first
    stream_sym[1::2] = second
    stream_take = np.empty(2 * Q, bool)
    stream_take[0::2] = take_first
    stream_take[1::2] = take_second
    copy = stream_sym[stream_take]
    # copy length per pair
    emit_per_pair = np.add.reduceat(n_emit, q_off[:-1]) if Q > 0 else np.zeros(P, np.int64)
    emit_per_pair = np.where(q_lens > 0, emit_per_pair, 0).astype(np.int64)
    c_off = np.zeros(P + 1, np.int64)
    c_off[1:] = np.cumsum(emit_per_pair)

    r_lens = np.maximum(r_lens, emit_per_pair)
    r_off = np.zeros(P + 1, np.int64)
    r_off[1:] = np.cumsum(r_lens)
    refs = _draw(rng, int(r_off[-1]), pi, A)
    slack = r_lens - emit_per_pair
    offset = (rng.random(P) * (slack + 1)).astype(np.int64)
    offset = np.minimum(offset, slack)
    # put the copies into refs: they occupy disjoint runs in pair order, so a
    # mask of the runs (from +1/-1 marks at their ends) takes them in order
    if c_off[-1] > 0:
        start = r_off[:-1] + offset
        marks = np.zeros(int(r_off[-1]) + 1, np.int8)
        np.add.at(marks, start, 1)
        np.add.at(marks, start + emit_per_pair, -1)
        refs[np.cumsum(marks[:-1], dtype=np.int8) > 0] = copy
    return queries, q_off, refs, r_off


def _concat(parts):
    qs, qo, rs, ro = [], [np.zeros(1, np.int64)], [], [np.zeros(1, np.int64)]
    qbase = 0
    rbase = 0
    for q, q_off, r, r_off in parts:
        qs.append(q)
        rs.append(r)
        qo.append(q_off[1:] + qbase)
        ro.append(r_off[1:] + rbase)
        qbase += int(q_off[-1])
        rbase += int(r_off[-1])
    return (np.concatenate(qs) if qs else np.zeros(0, np.uint8), np.concatenate(qo),
            np.concatenate(rs) if rs else np.zeros(0, np.uint8), np.concatenate(ro))


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

WORKLOADS = ("dna_small", "dna_large", "protein", "mixed", "serving")
_CHUNK = 50_000


def _uniform_lengths(rng, n, lo, hi):
    return rng.integers(lo, hi + 1, size=n).astype(np.int64)


def mixed_lengths(rng, n):
    """Query length round(LogNormal(ln 150, 0.8)) clipped to [32, 1024] with
    probability 0.95, else U{1024..2048}; reference round(q * U[1.5, 3])."""
    q = np.rint(rng.lognormal(math.log(150.0), 0.8, size=n))
    q = np.clip(q, 32, 1024)
    long_mask = rng.random(n) >= 0.95
    q[long_mask] = rng.integers(1024, 2049, size=int(long_mask.sum()))
    q = q.astype(np.int64)
    r = np.rint(q * rng.uniform(1.5, 3.0, size=n)).astype(np.int64)
    return q, r


def make_workload(name: str, n_pairs: Optional[int] = None, seed: Optional[int] = None,
                  scheme_seed: Optional[int] = None) -> Batch:
    """Generate one of the named workloads, optionally truncated to the first
    ``n_pairs`` draws (the draw order is fixed by the seed, so a smaller
    n_pairs gives a prefix-like sample of the same distribution).  The protein
    matrix and residue frequencies are drawn from ``scheme_seed`` (default:
    the same seed), so many batches can share one scoring scheme."""
    idx = WORKLOADS.index(name)
    seed = BASE_SEED + idx if seed is None else seed
    scheme_seed = seed if scheme_seed is None else scheme_seed
    rng = np.random.default_rng(seed)
    dna = dna_scheme()
    prot = protein_scheme(scheme_seed)
    pi_prot = protein_frequencies(scheme_seed)

    if name == "dna_small":
        P = 1000 if n_pairs is None else n_pairs
        q, qo, r, ro = mutate_embed(rng, _uniform_lengths(rng, P, 50, 150),
                                    _uniform_lengths(rng, P, 100, 300), 0.10, 0.02, None, 4)
        return Batch(q, qo, r, ro, np.zeros(P, np.uint8), [dna], name, seed)
    if name == "dna_large":
        P = 200_000 if n_pairs is None else n_pairs
        parts = []
        for c0 in range(0, P, _CHUNK):
            c = min(_CHUNK, P - c0)
            parts.append(mutate_embed(rng, _uniform_lengths(rng, c, 100, 256),
                                      _uniform_lengths(rng, c, 200, 600), 0.10, 0.02, None, 4))
        q, qo, r, ro = _concat(parts)
        return Batch(q, qo, r, ro, np.zeros(P, np.uint8), [dna], name, seed)
    if name == "protein":
        P = 100_000 if n_pairs is None else n_pairs
        parts = []
        for c0 in range(0, P, _CHUNK):
            c = min(_CHUNK, P - c0)
            parts.append(mutate_embed(rng, _uniform_lengths(rng, c, 100, 500),
                                      _uniform_lengths(rng, c, 200, 1000), 0.30, 0.03, pi_prot, 20))
        q, qo, r, ro = _concat(parts)
        return Batch(q, qo, r, ro, np.zeros(P, np.uint8), [prot], name, seed)
    if name in ("mixed", "serving"):
        P = 1_000_000 if n_pairs is None else n_pairs
        parts = []
        sids = []
        for c0 in range(0, P, _CHUNK):
            c = min(_CHUNK, P - c0)
            is_prot = rng.random(c) < 0.20
            ql, rl = mixed_lengths(rng, c)
            # draw DNA and protein sub-batches, then interleave back in draw order
            d_idx = np.flatnonzero(~is_prot)
            p_idx = np.flatnonzero(is_prot)
            dq, dqo, dr, dro = mutate_embed(rng, ql[d_idx], rl[d_idx], 0.10, 0.02, None, 4)
            pq, pqo, pr, pro = mutate_embed(rng, ql[p_idx], rl[p_idx], 0.30, 0.03, pi_prot, 20)
            parts.append(_interleave(is_prot, (dq, dqo, dr, dro), (pq, pqo, pr, pro)))
            sids.append(is_prot.astype(np.uint8))
        q, qo, r, ro = _concat(parts)
        return Batch(q, qo, r, ro, np.concatenate(sids), [dna, prot], name, seed)
    raise ValueError(name)


def _interleave(is_b, a, b):
    """Merge two packed sub-batches back into the order given by mask is_b."""
    aq, aqo, ar, aro = a
    bq, bqo, br, bro = b
    P = is_b.size
    ql = np.zeros(P, np.int64)
    rl = np.zeros(P, np.int64)
    ql[~is_b] = np.diff(aqo)
    ql[is_b] = np.diff(bqo)
    rl[~is_b] = np.diff(aro)
    rl[is_b] = np.diff(bro)
    qo = np.zeros(P + 1, np.int64)
    qo[1:] = np.cumsum(ql)
    ro = np.zeros(P + 1, np.int64)
    ro[1:] = np.cumsum(rl)
    # each sub-batch's residues keep their order in the merged layout, so
    # a per-residue owner mask places them
    q = np.empty(int(qo[-1]), np.uint8)
    r = np.empty(int(ro[-1]), np.uint8)
    q_owner = np.repeat(is_b, ql)
    r_owner = np.repeat(is_b, rl)
    q[~q_owner] = aq
    q[q_owner] = bq
    r[~r_owner] = ar
    r[r_owner] = br
    return q, qo, r, ro


@dataclasses.dataclass
class Request:
    arrival_s: float
    batch: Batch


def serving_requests(n_requests: int, seed: Optional[int] = None, max_pairs: int = 5000) -> List[Batch]:
    """The request bodies of a serving stream: each a batch of U{1..max_pairs}
    pairs from the mixed draw with its own seed; all share one protein
    scheme, drawn from the stream's base seed."""
    base = BASE_SEED + WORKLOADS.index("serving") if seed is None else seed
    rng = np.random.default_rng(base)
    sizes = rng.integers(1, max_pairs + 1, size=n_requests)
    return [make_workload("mixed", n_pairs=int(s), seed=base * 1000 + k, scheme_seed=base)
            for k, s in enumerate(sizes)]


def poisson_arrivals(n: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def serving_stream(offered_cells_per_ms: float, n_requests: int, seed: Optional[int] = None,
                   max_pairs: int = 5000) -> List[Request]:
    """Poisson stream of requests at the offered load.  Each request is a
    batch of U{1..max_pairs} pairs from the mixed draw with its own seed; the
    arrival rate is the offered load divided by the mean cells per request."""
    base = BASE_SEED + WORKLOADS.index("serving") if seed is None else seed
    batches = serving_requests(n_requests, base, max_pairs)
    mean_cells = float(np.mean([b.cells() for b in batches]))
    lam = offered_cells_per_ms * 1e3 / mean_cells  # requests per second
    t = poisson_arrivals(n_requests, lam, base + 1)
    return [Request(float(t[k]), batches[k]) for k in range(n_requests)]


# ---- database search: one query against many references ---------------------

@dataclasses.dataclass
class SearchSet:
    """One query and a set of references (the flat layout of sw_search)."""

    query: np.ndarray
    refs: np.ndarray
    r_off: np.ndarray
    scheme: Scheme
    name: str = ""
    seed: int = 0
    homolog: Optional[np.ndarray] = None   # bool [n_refs]: the reference embeds a copy of the query

    @property
    def n_refs(self) -> int:
        return int(self.r_off.shape[0] - 1)

    def cells(self) -> int:
        return int(self.query.size) * int(self.r_off[-1] - self.r_off[0])

    def as_batch(self, index=None) -> Batch:
        """The same pairs as a Batch (the query copied for each pair), or the
        pairs `index` only."""
        idx = np.arange(self.n_refs) if index is None else np.asarray(index, dtype=np.int64)
        n = self.query.size
        q = np.tile(self.query, idx.size)
        qo = np.arange(idx.size + 1, dtype=np.int64) * n
        lens = (self.r_off[idx + 1] - self.r_off[idx]).astype(np.int64)
        ro = np.zeros(idx.size + 1, np.int64)
        np.cumsum(lens, out=ro[1:])
        r = np.concatenate([self.refs[self.r_off[i]:self.r_off[i + 1]] for i in idx]) if idx.size else \
            np.zeros(0, np.uint8)
        return Batch(q, qo, r.astype(np.uint8), ro, np.zeros(idx.size, np.uint8), [self.scheme],
                     self.name + "[batch]", self.seed)


SEARCHES = ("search_protein", "search_dna")


def make_search(name: str, n_refs: Optional[int] = None, seed: Optional[int] = None) -> SearchSet:
    """A database search: one query against references of which 1% embed a
    mutated copy of it (the homologues a search is for) and the rest are
    unrelated sequences of the same residue distribution.
      search_protein: query of 400 residues, 200,000 references of
        U{100..1000}, the protein scheme and mutation rates of "protein";
      search_dna: query of 256 residues, 1,000,000 references of U{200..600},
        the DNA scheme and mutation rates of "dna_large"."""
    idx = SEARCHES.index(name)
    seed = BASE_SEED + 100 + idx if seed is None else seed
    rng = np.random.default_rng(seed)
    if name == "search_protein":
        n_q, P, lo, hi, A = 400, 200_000, 100, 1000, 20
        scheme, pi, p_sub, p_indel = protein_scheme(seed), protein_frequencies(seed), 0.30, 0.03
    else:
        n_q, P, lo, hi, A = 256, 1_000_000, 200, 600, 4
        scheme, pi, p_sub, p_indel = dna_scheme(), None, 0.10, 0.02
    P = P if n_refs is None else n_refs
    query = _draw(rng, n_q, pi, A)
    r_len = _uniform_lengths(rng, P, lo, hi)
    homolog = rng.random(P) < 0.01
    parts_r = []
    r_off = np.zeros(P + 1, np.int64)
    # homologues: mutated embeddings of the query
    h_idx = np.flatnonzero(homolog)
    _, _, hr, hro = mutate_embed(rng, np.full(h_idx.size, n_q), r_len[h_idx], p_sub, p_indel, pi, A,
                                 queries=np.tile(query, h_idx.size))
    lens = r_len.astype(np.int64).copy()
    lens[h_idx] = np.diff(hro)
    r_off[1:] = np.cumsum(lens)
    refs = _draw(rng, int(r_off[-1]), pi, A)
    for k, i in enumerate(h_idx):
        refs[r_off[i]:r_off[i + 1]] = hr[hro[k]:hro[k + 1]]
    return SearchSet(query, refs, r_off, scheme, name, seed, homolog)
