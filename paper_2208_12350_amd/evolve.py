"""Evolutionary search over the library's launch parameters, and the
analysis of the edits it finds.

This applies the paper's method to this project's own kernels at the level
of their parameters (not of their code): the evolutionary loop of Section
II-A (a population of program variants made by mutation and crossover from
one starting program, validated on test inputs, selected by a fitness
measure, iterated), with the search settings of Section III-E (elitism,
per-individual crossover and mutation probabilities), and the analysis of
Section V: weak-edit elimination (Algorithm 1), the split into independent
and epistatic edits (Algorithm 2), and the exhaustive evaluation of the
subsets of the epistatic edits.

An *edit* sets one parameter of a configuration of libswalign:

* ``("route", lo, hi, W, R)``: queries of lo+1 .. hi residues on the packed
  int16 path go to the sweep shape of W lanes x R rows per lane;
* ``("opt", name, value)``: a library option (``streams``, ``mode``,
  ``graph``, ``colpath``, ``pairtable``, ``chunk``, ``families``).

A genome is a list of edits, applied in order to the default configuration
(later edits override earlier ones where they overlap).  A configuration
*fails* when it cannot be built (a shape that does not cover its rows) or
when its results differ from the default configuration's: every variant must
reproduce the reference results exactly, as in the paper's validation step.
Fitness is the wall time of one sw_align_batch call on the batch (lower is
better; the median of a few timed calls after a warm-up call).

The search and the analysis only see a ``measure(edits) -> ms or None``
function, so they are tested on the CPU with synthetic fitness functions;
``LibraryFitness`` measures real configurations on the GPU.
"""
from __future__ import annotations

import json
import random
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

Edit = Tuple
Genome = List[Edit]
Measure = Callable[[Sequence[Edit]], Optional[float]]

BUCKET = 16
MAX_QUERY = 2048
OPTION_VALUES = {"streams": (1, 2, 3, 4), "mode": (0, 1), "graph": (0, 1), "colpath": (0, 1), "pairtable": (0, 1),
                 "chunk": (128, 64), "families": (0, 1)}


# ---- configurations -------------------------------------------------------------

def apply_edits(default_route: Sequence[Tuple[int, int]], edits: Sequence[Edit],
                shapes: Sequence[Tuple[int, int]]):
    """The configuration an edit list gives: (per-bucket shapes, options),
    or None if an edit is invalid (unknown shape, or one that does not cover
    the rows routed to it)."""
    route = list(default_route)
    opts: Dict[str, int] = {}
    known = set(shapes)
    for e in edits:
        if e[0] == "route":
            _, lo, hi, W, R = e
            if (W, R) not in known or W * R < hi or lo < 0 or hi > MAX_QUERY or lo >= hi:
                return None
            for k in range(lo // BUCKET, hi // BUCKET):
                route[k] = (W, R)
        elif e[0] == "opt":
            _, name, value = e
            if name not in OPTION_VALUES or value not in OPTION_VALUES[name]:
                return None
            opts[name] = value
        else:
            return None
    return route, opts


def tuning_string(route: Sequence[Tuple[int, int]], opts: Dict[str, int]) -> str:
    """sw_create's tuning string for a configuration."""
    table = []
    for k, (W, R) in enumerate(route):
        hi = BUCKET * (k + 1)
        if table and (table[-1][1], table[-1][2]) == (W, R):
            table[-1] = (hi, W, R)
        else:
            table.append((hi, W, R))
    parts = ["route16=" + "/".join("%dx%d@%d" % (W, R, hi) for hi, W, R in table)]
    parts += ["%s=%d" % (k, v) for k, v in sorted(opts.items())]
    return ";".join(parts)


# ---- the evolutionary search ------------------------------------------------------

def random_edit(rng: random.Random, shapes: Sequence[Tuple[int, int]], max_span: int = 64,
                weights: Optional[Sequence[float]] = None) -> Edit:
    """A random parameter edit: mostly routing edits over a short range of
    16-row buckets to a shape that covers at least the range's first bucket
    (so some edits are invalid, as random mutations are), else an option.
    The range starts at a bucket drawn with `weights` (e.g. the workload's
    query-length histogram; uniform when None)."""
    if rng.random() < 0.8:
        nb = MAX_QUERY // BUCKET
        a = rng.choices(range(nb), weights=weights)[0] if weights is not None else rng.randrange(nb)
        # spans from one bucket to max_span, short ones more often
        b = min(nb, a + min(max_span, int(2 ** rng.uniform(0, 6.01))))
        lo, hi = a * BUCKET, b * BUCKET
        fit = [s for s in shapes if s[0] * s[1] >= lo + BUCKET]
        W, R = rng.choice(fit)
        return ("route", lo, hi, W, R)
    name = rng.choice(sorted(OPTION_VALUES))
    return ("opt", name, rng.choice(OPTION_VALUES[name]))


def mutate(genome: Genome, rng: random.Random, shapes, weights=None, max_span: int = 64) -> Genome:
    """One mutation: insert a new edit, delete one, or replace one."""
    g = list(genome)
    op = rng.random()
    if not g or op < 0.5:
        g.insert(rng.randint(0, len(g)), random_edit(rng, shapes, max_span, weights))
    elif op < 0.75:
        del g[rng.randrange(len(g))]
    else:
        g[rng.randrange(len(g))] = random_edit(rng, shapes, max_span, weights)
    return g


def crossover(a: Genome, b: Genome, rng: random.Random) -> Tuple[Genome, Genome]:
    """One-point crossover of two edit lists."""
    ca, cb = rng.randint(0, len(a)), rng.randint(0, len(b))
    return a[:ca] + b[cb:], b[:cb] + a[ca:]


class Evaluator:
    """Caches measurements by variant, as GEVO caches program variants: by
    the configuration an edit list builds when the measure provides
    ``key(edits)`` (so edit lists that build the same configuration, e.g.
    one that sets an option to its default, share one measurement), else by
    the edit list."""

    def __init__(self, measure: Measure):
        self.measure = measure
        self.keyfn = getattr(measure, "key", None)
        self.cache: Dict[str, Optional[float]] = {}
        self.calls = 0

    def __call__(self, edits: Sequence[Edit]) -> Optional[float]:
        key = self.keyfn(edits) if self.keyfn else json.dumps(list(map(list, edits)))
        if key not in self.cache:
            self.calls += 1
            self.cache[key] = self.measure(edits)
        return self.cache[key]


def evolve(measure: Measure, shapes, population: int = 32, generations: int = 10, elite: int = 4,
           p_crossover: float = 0.8, p_mutation: float = 0.3, tournament: int = 2, seed: int = 0,
           weights: Optional[Sequence[float]] = None, max_span: int = 64,
           log: Optional[Callable[[str], None]] = None):
    """Evolve edit lists against `measure` (lower is better; None = the
    variant fails).  Each generation keeps the `elite` best, then fills the
    population with children of tournament-selected parents: crossover with
    probability p_crossover per pair, then one mutation with probability
    p_mutation per child.  Returns (best genome, its ms, history of the best
    ms per generation, evaluator)."""
    rng = random.Random(seed)
    ev = measure if isinstance(measure, Evaluator) else Evaluator(measure)
    pop: List[Genome] = [[]]
    while len(pop) < population:
        g: Genome = []
        for _ in range(rng.randint(1, 3)):
            g = mutate(g, rng, shapes, weights, max_span)
        pop.append(g)

    def fitness(g):
        t = ev(g)
        return float("inf") if t is None else t

    history = []
    for gen in range(generations + 1):
        scored = sorted(pop, key=fitness)
        best = scored[0]
        history.append(fitness(best))
        if log:
            valid = sum(1 for g in pop if ev(g) is not None)
            log("generation %d: best %.4f ms (%d edits), %d/%d valid, %d measurements"
                % (gen, history[-1], len(best), valid, len(pop), ev.calls))
        if gen == generations:
            break
        nxt = [list(g) for g in scored[:elite]]

        def pick():
            cands = [rng.choice(scored) for _ in range(tournament)]
            return min(cands, key=fitness)
        while len(nxt) < population:
            a, b = pick(), pick()
            if rng.random() < p_crossover:
                a, b = crossover(a, b, rng)
            for child in (a, b):
                if rng.random() < p_mutation:
                    child = mutate(child, rng, shapes, weights, max_span)
                if len(nxt) < population:
                    nxt.append(list(child))
        pop = nxt
    return best, fitness(best), history, ev


# ---- the edit analysis ------------------------------------------------------------

def _without(edits: Sequence[Edit], drop: Sequence[Edit]) -> Genome:
    out, gone = [], list(drop)
    for e in edits:
        if e in gone:
            gone.remove(e)
        else:
            out.append(e)
    return out


def weak_edits(edits: Sequence[Edit], measure: Measure, threshold: float = 0.01) -> Genome:
    """Algorithm 1: an edit is weak when, in the context of the edits not yet
    found weak, dropping it changes the performance f = 1 / time by less than
    `threshold`:  (f(S - weaks) - f(S - weaks - e)) / f(S - weaks - e) <
    threshold.  An edit whose removal makes the configuration fail is not
    weak."""
    weaks: Genome = []
    for e in edits:
        t_with = measure(_without(edits, weaks))
        t_without = measure(_without(edits, weaks + [e]))
        if t_with is None or t_without is None:
            continue
        gain = (1.0 / t_with - 1.0 / t_without) / (1.0 / t_without)
        if gain < threshold:
            weaks.append(e)
    return weaks


def split_independent(edits: Sequence[Edit], measure: Measure, tolerance: float = 0.01):
    """Algorithm 2: an edit is independent when it can be applied alone and
    removed from the rest without failing, and its relative time saving alone
    on the original, (t(none) - t(e)) / t(none), agrees within `tolerance`
    with its saving in the context of the remaining edits,
    (t(S - Indep - e) - t(S - Indep)) / t(S - Indep - e).  Whatever remains
    is epistatic.  Returns (independent, epistatic, per-edit savings)."""
    indep: Genome = []
    t0 = measure([])
    savings = {}
    for e in edits:
        t_alone = measure([e])
        t_rest = measure(_without(edits, indep + [e]))
        if t0 is None or t_alone is None or t_rest is None:
            continue
        incr = (t0 - t_alone) / t0
        t_ctx = measure(_without(edits, indep))
        if t_ctx is None:
            continue
        decr = (t_rest - t_ctx) / t_rest
        savings[json.dumps(list(e))] = (incr, decr)
        if abs(incr - decr) <= tolerance:
            indep.append(e)
    return indep, _without(edits, indep), savings


def subset_times(edits: Sequence[Edit], measure: Measure, max_edits: int = 10):
    """Time of every subset of a small edit set (applied to the original, in
    the set's order): the exhaustive search for interacting subgroups."""
    n = len(edits)
    if n > max_edits:
        raise ValueError("%d edits: too many subsets" % n)
    out = []
    for mask in range(1 << n):
        sub = [edits[k] for k in range(n) if mask >> k & 1]
        out.append((mask, measure(sub)))
    return out


def analyse(edits: Sequence[Edit], measure: Measure, threshold: float = 0.01, tolerance: float = 0.01,
            max_subset_edits: int = 10):
    """Weak-edit elimination, then the independent / epistatic split, then
    the subsets of the epistatic edits (when there are few)."""
    weaks = weak_edits(edits, measure, threshold)
    strong = _without(edits, weaks)
    indep, epi, savings = split_independent(strong, measure, tolerance)
    subsets = subset_times(epi, measure) if 0 < len(epi) <= max_subset_edits else []
    return {"weak": weaks, "strong": strong, "independent": indep, "epistatic": epi, "savings": savings,
            "epistatic_subsets": subsets, "t_original": measure([]), "t_all": measure(list(edits)),
            "t_strong": measure(strong)}


# ---- measuring real configurations on the GPU --------------------------------------

class LibraryFitness:
    """measure(edits): build the configuration, align the device batch with
    it, check the results against the default configuration's, and return
    the median wall time in ms of `repeats` calls after a warm-up call (None
    when the configuration fails)."""

    def __init__(self, dbatch, device: int = 0, repeats: int = 3):
        import torch
        from .binding import Aligner
        self.db = dbatch
        self.device = device
        self.repeats = repeats
        probe = Aligner(device)
        self.shapes = [(w, r) for p, w, r in probe.shapes() if p == 16]
        table = probe.routing(16)
        probe.close()
        self.default_route = []
        prev = 0
        for hi, W, R in table:
            self.default_route += [(W, R)] * ((hi - prev) // BUCKET)
            prev = hi
        # forward cells per 16-row bucket of query length: where routing
        # edits matter
        ql = (dbatch.q_off[1:] - dbatch.q_off[:-1]).clamp(1, MAX_QUERY).cpu()
        rl = (dbatch.r_off[1:] - dbatch.r_off[:-1]).cpu().double()
        hist = torch.bincount((ql - 1) // BUCKET, weights=ql.double() * rl, minlength=MAX_QUERY // BUCKET)
        total = float(hist.sum()) or 1.0
        self.weights = [float(h) / total + 1e-4 for h in hist]
        self.out = torch.empty((dbatch.n_pairs, 5), dtype=torch.int32, device="cuda:%d" % device)
        self.ref_out = None
        if self._run("", check=False) is None:
            raise RuntimeError("the default configuration failed")

    def _run(self, tuning, check=True):
        import torch
        from .binding import Aligner, SwError
        try:
            al = Aligner(self.device, tuning or None)
        except RuntimeError:
            return None
        try:
            al.align(self.db, self.out)
            torch.cuda.synchronize()
            if check and not torch.equal(self.out, self.ref_out):
                return None
            ts = []
            for _ in range(self.repeats):
                t = time.perf_counter()
                al.align(self.db, self.out)
                ts.append((time.perf_counter() - t) * 1e3)
            if not check:
                self.ref_out = self.out.clone()
            ts.sort()
            return ts[len(ts) // 2]
        except SwError:
            return None
        finally:
            al.close()

    DEFAULT_OPTIONS = {"streams": 4, "mode": 1, "graph": 1, "colpath": 1, "pairtable": 1, "chunk": 128, "families": 1}

    def key(self, edits: Sequence[Edit]) -> str:
        """The configuration an edit list builds, with options at their
        default values dropped ("fail" for an invalid one)."""
        cfg = apply_edits(self.default_route, edits, self.shapes)
        if cfg is None:
            return "fail"
        route, opts = cfg
        return tuning_string(route, {k: v for k, v in opts.items() if self.DEFAULT_OPTIONS.get(k) != v})

    def noise(self, n: int = 5) -> float:
        """Spread (max - min) / median of n measurements of the default
        configuration, each with a fresh handle."""
        ts = sorted(self._run("") for _ in range(n))
        return (ts[-1] - ts[0]) / ts[len(ts) // 2]

    def __call__(self, edits: Sequence[Edit]) -> Optional[float]:
        cfg = apply_edits(self.default_route, edits, self.shapes)
        if cfg is None:
            return None
        return self._run(tuning_string(*cfg))


def main(argv=None):
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="evolutionary search over libswalign's launch parameters")
    ap.add_argument("--workload", default="dna_large")
    ap.add_argument("--n-pairs", type=int, default=None)
    ap.add_argument("--population", type=int, default=24)
    ap.add_argument("--generations", type=int, default=8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--repeats", type=int, default=3)
    args = ap.parse_args(argv)
    from . import workloads as W
    from .binding import DeviceBatch
    log = lambda s: print(s, file=sys.stderr, flush=True)
    batch = W.make_workload(args.workload, n_pairs=args.n_pairs)
    db = DeviceBatch.from_host(batch, "cuda:0")
    fit = LibraryFitness(db, repeats=args.repeats)
    ev = Evaluator(fit)
    noise = fit.noise()
    log("measurement spread of the default configuration: %.1f%%" % (100 * noise))
    t0 = time.time()
    best, best_ms, history, ev = evolve(ev, fit.shapes, population=args.population,
                                        generations=args.generations, seed=args.seed, weights=fit.weights,
                                        log=log)
    t_search = time.time() - t0
    # the paper's 1% thresholds, raised to the measurement spread
    thr = max(0.01, noise)
    log("analysing %d edits (threshold %.1f%%) ..." % (len(best), 100 * thr))
    rep = analyse(best, ev, threshold=thr, tolerance=thr)
    res = {"workload": args.workload, "pairs": batch.n_pairs, "population": args.population,
           "generations": args.generations, "measurements": ev.calls, "search_s": round(t_search, 1),
           "t_default_ms": ev([]), "t_best_ms": best_ms, "history_ms": history, "noise": round(noise, 4),
           "threshold": round(thr, 4),
           "best_edits": best, "best_tuning": tuning_string(*apply_edits(fit.default_route, best, fit.shapes)),
           "analysis": {k: v for k, v in rep.items() if k != "savings"},
           "savings": rep["savings"]}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
