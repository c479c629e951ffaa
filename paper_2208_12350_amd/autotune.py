"""Autotuner for the sweep routing: which shape (lanes per pair W, query rows
per lane R) aligns which query lengths, i.e. the group width, the tile
height and the bin edges of the length binning.

Two steps:

1. ``measure_rates``: every compiled shape of a precision sweeps a
   homogeneous probe batch (queries of exactly W*R residues, references of
   a given length) with a routing that sends the probe to that shape; the
   per-launch HIP-event time of the forward sweep gives the shape's rate in
   lane-row slots per millisecond.  A slot is one (row, column) position a
   lane group sweeps, padding included: a pair of n rows and m columns on
   shape (W, R) costs W * R * (m + W - 1) slots.
2. ``choose_routing``: for each 16-row bucket of query lengths, the covering
   shape with the least predicted time for the pairs of that bucket in a
   sample of the workload, time = slots / rate.  Pure host arithmetic, so it
   is tested without a GPU.

3. ``pick_by_timing``: the rate model ignores the critical path of the
   longest pairs, which bounds small batches and the tail of large ones; so
   the model's table and variants that put long queries on cooperative
   256-lane groups (``candidate_tables``) are each timed on the batch
   itself, and the fastest wins.
4. The tile width: the winning table is timed again with the 16- and
   32-lane shapes streaming the reference in tiles of 64 steps instead of
   128 (fewer prefetch registers per lane, twice as many tile boundaries),
   and the faster tile is kept.

The result is a routing table [(rows_max, W, R), ...] for
``Aligner.set_routing`` and a tile width, or, as a string
(``tuning_string``), for the tuning argument of ``sw_create``.  Results
never depend on the routing or the tile; only speed does.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

MAX_QUERY = 2048
BUCKET = 16

Shape = Tuple[int, int]          # (W, R)
Table = List[Tuple[int, int, int]]


def slots(m: np.ndarray, shape: Shape) -> np.ndarray:
    """Lane-row slots a group of shape (W, R) sweeps for pairs with
    references of m residues (their query must fit in W * R rows)."""
    W, R = shape
    return W * R * (np.asarray(m, dtype=np.float64) + W - 1)


def choose_routing(q_len: np.ndarray, r_len: np.ndarray, rates: Dict[Shape, float],
                   default_m: float = 512.0) -> Table:
    """Routing table minimising the predicted sweep time of the sample
    (q_len, r_len) under per-shape rates (slots per ms).  Buckets with no
    sample pair use a reference length of twice the bucket's rows plus 64
    (or ``default_m``, whichever is larger)."""
    if not rates:
        raise ValueError("no shape rates")
    q_len = np.asarray(q_len, dtype=np.int64)
    r_len = np.asarray(r_len, dtype=np.int64)
    keep = (q_len > 0) & (r_len > 0)
    q_len, r_len = q_len[keep], r_len[keep]
    bucket = (np.minimum(q_len, MAX_QUERY) - 1) // BUCKET
    choice = []
    for k in range(MAX_QUERY // BUCKET):
        rows = BUCKET * (k + 1)
        m = r_len[bucket == k]
        if m.size == 0:
            m = np.array([max(default_m, 2.0 * rows + 64)])
        best, best_t = None, None
        for shape, rate in rates.items():
            W, R = shape
            if W * R < rows or rate <= 0:
                continue
            t = float(np.sum(slots(m, shape))) / rate
            if best is None or t < best_t or (t == best_t and W * R < best[0] * best[1]):
                best, best_t = shape, t
        if best is None:
            raise ValueError("no measured shape covers %d rows" % rows)
        choice.append(best)
    return merge(choice)


def merge(choice: Sequence[Shape]) -> Table:
    """Per-bucket shapes -> routing table of merged runs."""
    table: Table = []
    for k, (W, R) in enumerate(choice):
        hi = BUCKET * (k + 1)
        if table and (table[-1][1], table[-1][2]) == (W, R):
            table[-1] = (hi, W, R)
        else:
            table.append((hi, W, R))
    return table


def expand(table: Table) -> List[Shape]:
    """Routing table -> the shape of every 16-row bucket."""
    out, prev = [], 0
    for hi, W, R in table:
        out.extend([(W, R)] * ((hi - prev) // BUCKET))
        prev = hi
    return out


def predicted_ms(q_len, r_len, table: Table, rates: Dict[Shape, float]) -> float:
    """Predicted sweep time of a sample under a routing table."""
    shapes = expand(table)
    q_len = np.asarray(q_len, dtype=np.int64)
    r_len = np.asarray(r_len, dtype=np.int64)
    keep = (q_len > 0) & (r_len > 0)
    q_len, r_len = q_len[keep], r_len[keep]
    bucket = (np.minimum(q_len, MAX_QUERY) - 1) // BUCKET
    total = 0.0
    for k, shape in enumerate(shapes):
        m = r_len[bucket == k]
        if m.size:
            total += float(np.sum(slots(m, shape))) / rates[shape]
    return total


def _probe_batch(W: int, R: int, m: int, n_pairs: int, seed: int, scheme):
    from . import workloads as WL
    rng = np.random.default_rng(seed)
    n = W * R
    A = scheme.alphabet
    q = rng.integers(0, A, size=n_pairs * n).astype(np.uint8)
    r = rng.integers(0, A, size=n_pairs * m).astype(np.uint8)
    q_off = np.arange(n_pairs + 1, dtype=np.int64) * n
    r_off = np.arange(n_pairs + 1, dtype=np.int64) * m
    return WL.Batch(q, q_off, r, r_off, np.zeros(n_pairs, np.uint8), [scheme], "probe", seed)


def dominant_scheme(batch):
    """The scheme of a batch that carries the most forward cells (its
    substitution scores decide which kernel variant the probes should time)."""
    cells = (batch.q_len().astype(np.int64) * batch.r_len().astype(np.int64))
    per = np.bincount(batch.scheme_id.astype(np.int64), weights=cells.astype(np.float64),
                      minlength=len(batch.schemes))
    return batch.schemes[int(np.argmax(per))]


def measure_rates(device: int = 0, precision: int = 16, m: int = 512, target_cells: float = 4e9,
                  repeats: int = 2, shapes: Optional[Sequence[Shape]] = None,
                  log=None, scheme=None) -> Dict[Shape, float]:
    """Slots per millisecond of the forward sweep of every compiled shape of
    `precision` (or of `shapes`), from per-launch HIP-event timing, on
    random sequences scored by `scheme` (default: the DNA scheme; a small
    alphabet runs the column-word kernels, a large one the table kernels)."""
    from . import workloads as WL
    scheme = scheme if scheme is not None else WL.dna_scheme()
    import torch
    from .binding import Aligner, DeviceBatch

    al = Aligner(device, timing=2, precision=32 if precision == 32 else 0)
    try:
        compiled = [(w, r) for p, w, r in al.shapes() if p == precision]
        todo = list(shapes) if shapes is not None else compiled
        big = max(compiled, key=lambda s: s[0] * s[1])
        rates: Dict[Shape, float] = {}
        for W, R in todo:
            ppw = (64 // W if W <= 64 else 1) * (2 if precision == 16 else 1)
            n_pairs = int(np.clip(target_cells / (W * R * m), 2048 * ppw // 4, 400_000))
            n_pairs -= n_pairs % ppw
            b = _probe_batch(W, R, m, n_pairs, seed=W * 1000 + R, scheme=scheme)
            db = DeviceBatch.from_host(b, "cuda:%d" % device)
            out = torch.empty((n_pairs, 5), dtype=torch.int32, device="cuda:%d" % device)
            table = [(W * R, W, R)]
            if W * R < MAX_QUERY:
                table.append((MAX_QUERY, big[0], big[1]))
            al.set_routing(precision, table)
            ms = []
            for k in range(repeats + 1):
                al.align(db, out)
                if k:
                    ms.append(sum(e["ms"] for e in al.bin_stats()
                                  if (e["pass"], e["precision"], e["lanes"], e["rows"]) == (0, precision, W, R)))
            t = float(np.median(ms))
            rates[(W, R)] = float(np.sum(slots(np.full(n_pairs, m), (W, R)))) / t
            if log:
                log("  shape %dx%d: %d pairs, %.3f ms, %.3g slots/ms" % (W, R, n_pairs, t, rates[(W, R)]))
            del db, out
        al.set_routing(precision, [])
        return rates
    finally:
        al.close()


def with_wide_groups(table: Table, rows_above: int, shapes: Sequence[Shape], width: int = 256) -> Table:
    """`table` with the queries longer than `rows_above` moved to the
    narrowest covering shape of `width` lanes (cooperative groups cut the
    latency of long pairs, which bounds small batches and batch tails)."""
    wide = sorted(r for w, r in shapes if w == width)
    if not wide:
        return list(table)
    choice = expand(table)
    for k in range(len(choice)):
        rows = BUCKET * (k + 1)
        if rows > rows_above:
            fit = [r for r in wide if width * r >= rows]
            if fit:
                choice[k] = (width, fit[0])
    return merge(choice)


def coarse_rates(rates: Dict[Shape, float], step: int) -> Dict[Shape, float]:
    """The shapes of `rates` whose rows per lane are a multiple of `step`
    (16-lane shapes below `step` and cooperative shapes are kept): a routing
    chosen among them has fewer bins."""
    return {s: v for s, v in rates.items() if s[0] > 64 or s[1] % step == 0 or (s[0] == 16 and s[1] < step)}


def candidate_tables(q_len, r_len, rates: Dict[Shape, float], shapes: Sequence[Shape],
                     builtin: Optional[Table] = None) -> Dict[str, Table]:
    """Routings worth timing on the real batch: the rate model's choice, the
    same with long queries on cooperative 256-lane groups, the model's choice
    among shapes with an even number and a multiple of four rows per lane
    ("coarse2", "coarse4": fewer bins, so shorter chains of launches per
    stream and fewer launch tails, for some padding), and the library's
    built-in routing."""
    model = choose_routing(q_len, r_len, rates)
    out = {"model": model}
    if builtin is not None and builtin != model:
        out["builtin"] = list(builtin)

    def add(name, t):
        if t not in out.values():
            out[name] = t

    for above in (512, 768, 1024):
        add("model+coop>%d" % above, with_wide_groups(model, above, shapes))
    for step in (2, 4):
        try:
            coarse = choose_routing(q_len, r_len, coarse_rates(rates, step))
        except ValueError:
            continue
        if coarse in out.values():
            continue
        add("coarse%d" % step, coarse)
        for above in (512, 768):
            add("coarse%d+coop>%d" % (step, above), with_wide_groups(coarse, above, shapes))
    return out


DEFAULT_TILE = 128
TILES = (128, 64)


def tuning_string(table: Table, tile: int = DEFAULT_TILE) -> str:
    """The sw_create tuning string of a routing table and tile width."""
    from .binding import routing_string
    s = routing_string(16, table)
    return s if tile == DEFAULT_TILE else s + ";chunk=%d" % tile


def pick_by_timing(dbatch, tables: Dict[str, Table], device: int = 0, repeats: int = 2, log=None,
                   tile: int = DEFAULT_TILE, options: str = ""):
    """Time one call per repeat of each routing (with reference tiles of
    `tile` steps, and the further tuning-string `options`) on the batch
    itself (graph replay, the headline configuration) and return (name,
    table, ms)."""
    import torch
    from .binding import Aligner
    out = torch.empty((dbatch.n_pairs, 5), dtype=torch.int32, device="cuda:%d" % device)
    best = None
    for name, table in tables.items():
        al = Aligner(device, tuning_string(table, tile) + (";" + options if options else ""))
        try:
            al.align(dbatch, out)
            torch.cuda.synchronize()
            ts = []
            for _ in range(repeats):
                t = time.perf_counter()
                al.align(dbatch, out)
                ts.append((time.perf_counter() - t) * 1e3)
        finally:
            al.close()
        ms = float(np.median(ts))
        if log:
            log("  candidate %s%s: %.3f ms" % (name, "" if tile == DEFAULT_TILE else " tile %d" % tile, ms))
        if best is None or ms < best[2]:
            best = (name, table, ms)
    return best


def tune_batch(batch, dbatch, device: int = 0, sample: int = 50000, repeats: int = 7, seed: int = 5, log=None,
               options: str = ""):
    """The routing a batch is timed with: shape rates measured on the batch's
    dominant scheme at its median reference length, the candidate tables of
    a seeded sample of its pairs, the fastest of them on the batch itself
    (median of `repeats` graph-replayed calls each), then the faster tile
    width for it; the calls are timed with the tuning-string `options`.
    Returns (name, table, candidates, tile)."""
    from .binding import Aligner
    rng = np.random.default_rng(seed)
    idx = rng.choice(batch.n_pairs, size=min(batch.n_pairs, sample), replace=False)
    ql, rl = batch.q_len()[idx], batch.r_len()[idx]
    m_med = int(np.clip(np.median(rl[rl > 0]) if np.any(rl > 0) else 512, 64, 4096))
    rates = measure_rates(device, 16, m=m_med, log=log, scheme=dominant_scheme(batch))
    probe = Aligner(device)
    try:
        builtin = probe.routing(16)
    finally:
        probe.close()
    cands = candidate_tables(ql, rl, rates, list(rates), builtin=builtin)
    name, table, ms = pick_by_timing(dbatch, cands, device, repeats=repeats, log=log, options=options)
    tile = DEFAULT_TILE
    for t in TILES:
        if t == DEFAULT_TILE:
            continue
        _, _, ms_t = pick_by_timing(dbatch, {name: table}, device, repeats=repeats, log=log, tile=t,
                                    options=options)
        if ms_t < ms:
            tile, ms = t, ms_t
    return name, table, cands, tile


def tune(q_len, r_len, device: int = 0, precision: int = 16, log=None, **kw):
    """Measure the shapes and choose a routing for the sample (q_len, r_len).
    Returns (table, rates, seconds spent)."""
    t0 = time.time()
    m = int(np.clip(np.median(np.asarray(r_len)[np.asarray(r_len) > 0]) if np.any(np.asarray(r_len) > 0) else 512,
                    64, 4096))
    rates = measure_rates(device, precision, m=m, log=log, **kw)
    table = choose_routing(q_len, r_len, rates)
    return table, rates, time.time() - t0
