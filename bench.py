#!/usr/bin/env python3
"""Benchmark: batched affine-gap Smith-Waterman (score + start/end) on one GPU.

One step = one sw_align_batch call over the whole workload, inputs already
resident in device memory: classification and length binning, the forward
sweep (score and end) and the reverse sweep (start) of every pair, and the
result scatter.  Prints ONE JSON line.

  python bench.py [--steps K] [--warmup W] [--workload dna_large] [--mode 0|1]

GCUPS = sum over pairs of n*m (forward cells, the usual definition) per
second of whole-call wall time, / 1e9.

The "cigar" object of the line times sw_align_cigar on the same batch: the
same results plus every pair's alignment path (SAM runs), with the roofline
of the box-sweep kernel that records the traceback choices.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic integer operations per DP cell: H-o (1), E (2), F (2),
# diag+s (1), max of four terms with 0 (3), running best / argmax (3).
OPS_PER_CELL = 12
# Alignment paths: per cell of a result box, the recurrence without the
# running best (9) plus the traceback choices it records: H from the
# diagonal? from F? (2), F opens? (1), E opens? (1).
PATH_OPS_PER_CELL = 13
# MI355X: 256 CUs x 64 lanes x 2.4 GHz of 32-bit VALU issue; packed 16-bit
# instructions carry two operations per lane.
VALU_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12
VALU_INT16X2_TOPS = 2 * VALU_INT32_TOPS


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stored_traffic(kernel, workload, sources_sha256=None, cells_per_launch=None):
    """HBM bytes per launch of `kernel` on `workload` from a committed
    counter summary (profiles/*_traffic.txt), or None when there is none or
    when the kernel sources (digest `sources_sha256`, by default that of the
    sweep kernels) changed since the counters were taken.  With
    `cells_per_launch` the stored bytes are rescaled by this run's cells per
    launch against the profiled run's (a routing the tuner picks anew may
    give the kernel a different share of the pairs; its bytes per cell stay)."""
    import glob
    import hashlib
    here = os.path.join(ROOT, "profiles")
    for path in sorted(glob.glob(os.path.join(here, "*_traffic.txt"))):
        kv = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel", "").replace("sw::", "") != kernel.replace("sw::", "") or kv.get("workload") != workload:
            continue
        if kv.get("sources_sha256") != (sources_sha256 or kernel_sources_sha256()):
            return None
        try:
            per_launch = float(kv["traffic_bytes_per_launch"])
            if cells_per_launch:
                per_launch *= float(cells_per_launch) / float(kv["cells_per_launch"])
            return round(per_launch)
        except (KeyError, ValueError, ZeroDivisionError):
            return None
    return None


def kernel_sources_sha256():
    """Digest of the HIP sources the sweep kernels (score and path sweeps)
    are built from."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2208_12350_amd", "csrc")
    for path in sorted(glob.glob(os.path.join(csrc, "*.h")) + glob.glob(os.path.join(csrc, "sw_queue*.hip")) +
                       glob.glob(os.path.join(csrc, "sw_trace.hip"))):
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# Worker threads the CPU baseline may use: the GPU machine grants one GPU's
# process 16 host threads, whatever the machine's core count is.
CPU_SHARE = 16


def cpu_baseline(batch, target_s=12.0, single_s=4.0):
    """Time the CPU oracle (as it stands) on bounded random samples of the
    same workload: on every host thread this process may use (at most the
    box's share of CPU_SHARE threads), and on one thread."""
    import numpy as np
    from oracle import oracle
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    cores = max(1, min(affinity, CPU_SHARE))
    rng = np.random.default_rng(2208)
    ql, rl = batch.q_len().astype(np.int64), batch.r_len().astype(np.int64)
    mean_cells = float(np.mean(ql * rl))

    def run(threads, seconds):
        # calibration sample, then a sample sized for about `seconds`
        n0 = min(batch.n_pairs, 20 * threads)
        idx = rng.choice(batch.n_pairs, size=n0, replace=False)
        t = time.perf_counter()
        oracle.align_batch(batch, index=idx, threads=threads)
        dt = max(time.perf_counter() - t, 1e-3)
        rate = float(np.sum(ql[idx] * rl[idx])) / dt
        n1 = int(min(batch.n_pairs, max(n0, seconds * rate / mean_cells)))
        idx = rng.choice(batch.n_pairs, size=n1, replace=False)
        t = time.perf_counter()
        oracle.align_batch(batch, index=idx, threads=threads)
        dt = time.perf_counter() - t
        cells = float(np.sum(ql[idx] * rl[idx]))
        return cells / dt / 1e9, n1, cells, dt

    v, n1, cells, dt = run(cores, target_s)
    v1, m1, cells1, dt1 = run(1, single_s)
    return {"value": round(v, 4), "unit": "GCUPS", "cores": cores, "kind": "oracle",
            "sample": "%d random pairs of the same workload (%.3g forward cells, forward+reverse "
                      "sweeps, %.1f s on %d threads)" % (n1, cells, dt, cores),
            "single_core": {"value": round(v1, 4), "sample": "%d random pairs (%.3g forward cells, %.1f s)"
                            % (m1, cells1, dt1)},
            "nproc": os.cpu_count(), "affinity": affinity,
            "build": "gcc " + " ".join(oracle.CFLAGS)}


def roofline_leg(args, db, out, tuning, mode, workload, steps):
    """The sweep launches as the timed call issues them (one kernel per
    shape family, or per bin), serialised on one stream with a HIP event
    pair around each (library option timing=2), and cells per launch from
    the device counters of the bins each launch swept.  The dominant kernel
    is the launch with the most device time; achieved = 12 * its cells / its
    average time."""
    from paper_2208_12350_amd.binding import Aligner
    alr = Aligner(0, tuning, mode=mode, graph=0, timing=2)
    per_launch = {}
    roof_steps = max(3, min(steps, 10))
    for k in range(roof_steps + 1):
        alr.align(db, out)
        if k:
            launches = {}
            for e in alr.bin_stats():
                if e["launch"] < 0:
                    continue
                # the bins of a family launch share its launch index and time
                fam = (e["family_hi"], e["family_lo"], e["family_waves"]) if e["family_hi"] else (e["rows"], 0, 0)
                key = (e["pass"], e["precision"], e["lanes"], fam, e["column"], e["tile"])
                acc = launches.setdefault((e["pass"], e["launch"]), [key, e["ms"], 0])
                acc[2] += e["cells"]
            for key, ms, cells in launches.values():
                acc = per_launch.setdefault(key, [0.0, 0, 0])
                acc[0] += ms; acc[1] += cells; acc[2] += 1
    alr.close()
    (dpass, dprec, dlanes, (drows, dlo, dwaves), dcol, dtile), (dms, dcells, dn) = max(per_launch.items(),
                                                                                      key=lambda kv: kv[1][0])
    launch_ms = dms / dn
    cells_per_launch = dcells / dn
    peak = VALU_INT16X2_TOPS if dprec == 16 else VALU_INT32_TOPS
    achieved = OPS_PER_CELL * cells_per_launch / (launch_ms / 1e3) / 1e12
    # every sweep launch of a step together, each at its own precision's peak
    fam_ms = sum(v[0] for v in per_launch.values()) / roof_steps
    fam_ops = OPS_PER_CELL * sum(v[1] for v in per_launch.values()) / roof_steps
    fam_peak_s = sum(OPS_PER_CELL * v[1] / roof_steps / ((VALU_INT16X2_TOPS if k[1] == 16 else VALU_INT32_TOPS) * 1e12)
                     for k, v in per_launch.items())
    direction = "true" if dpass else "false"
    if dlo:
        # family kernel: <precision, lanes, reverse, score source, waves per
        # SIMD, reference tile, rows largest first>
        kernel_name = "sw::sw_family_kernel<%d, %d, %s, %d, %d, %d, %s>" % (
            dprec, dlanes, direction, dcol, dwaves, dtile, ", ".join(str(r) for r in range(drows, dlo - 1, -1)))
    elif dlanes > 64:
        kernel_name = "sw::sw_coop_kernel<%d, %s>" % (drows, direction)
    elif dcol == 3:
        kernel_name = "sw::sw_qprof_kernel<%d, %d>" % (dlanes, drows)
    elif dcol == 2:
        kernel_name = ("sw::sw_ptab_kernel<%d, %d, %s>" % (dlanes, drows, direction) if dtile == 128 else
                       "sw::sw_ptab_chunk_kernel<%d, %d, %s, %d>" % (dlanes, drows, direction, dtile))
    elif dtile == 128:
        kernel_name = "sw::sw_queue_kernel<%d, %d, %d, %s, %s>" % (dprec, dlanes, drows, direction,
                                                                  "true" if dcol else "false")
    else:
        kernel_name = "sw::sw_queue_chunk_kernel<%d, %d, %d, %s, %s, %d>" % (
            dprec, dlanes, drows, direction, "true" if dcol else "false", dtile)
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 2),
            "unit": "Tops/s", "frac": round(achieved / peak, 4),
            "traffic": stored_traffic(kernel_name, workload, cells_per_launch=cells_per_launch),
            "kernel": kernel_name, "launches": dn, "launch_ms": round(launch_ms, 4),
            "cells_per_launch": int(cells_per_launch), "ops_per_cell": OPS_PER_CELL,
            "all_sweeps": {"ms": round(fam_ms, 3), "achieved": round(fam_ops / (fam_ms / 1e3) / 1e12, 3),
                           "frac": round(fam_peak_s / (fam_ms / 1e3), 4)}}


def cigar_leg(args, db, out, ref_out, tuning, score_ms, workload):
    """sw_align_cigar on the same batch: results plus every pair's path.
    GCUPS counts forward cells per second of whole-call wall time, as the
    headline does.  The box sweeps' kernels are then timed per launch (the
    library's timing=2, launches serialised) for their roofline:
    PATH_OPS_PER_CELL per box cell against the int32 VALU peak."""
    import numpy as np
    import torch
    from paper_2208_12350_amd.binding import Aligner
    al = Aligner(0, tuning)
    res = al.align_cigar(db, out=out)
    torch.cuda.synchronize()
    steps = max(2, min(args.steps, 5))
    t0 = time.perf_counter()
    for _ in range(steps):
        al.align_cigar(db, out=res[0], cigar_off=res[1], cigar=res[2], cigar_len=res[3])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    assert torch.equal(out, ref_out), "the paths call disagrees with the headline run"
    fwd = al.stats()[0]
    box_cells, rec_bytes, chunks, _, _ = al.cigar_stats()
    al.close()
    alt = Aligner(0, tuning, timing=2)
    sweep_ms, walk_ms, per_bin = [], [], {}
    reps = 3
    for k in range(reps):
        alt.align_cigar(db, out=res[0], cigar_off=res[1], cigar=res[2], cigar_len=res[3])
        _, _, _, sm, wm = alt.cigar_stats()
        sweep_ms.append(sm); walk_ms.append(wm)
        # the bins of one launch (a family launch sweeps several) share its time
        launches_of_call = {}
        for e in alt.bin_stats():
            if e["pass"] == 2:
                rows = (e["family_hi"], e["family_lo"]) if e["family_hi"] else (e["rows"], 0)
                acc = launches_of_call.setdefault(e["launch"], [(e["precision"], e["lanes"], rows, e["column"]),
                                                                e["ms"], 0, 0])
                acc[2] += e["cells"]; acc[3] += e["pairs"]
        for key, ms, cells, pairs in launches_of_call.values():
            if pairs:
                acc = per_bin.setdefault(key, [0.0, 0])
                acc[0] += ms; acc[1] += cells
    alt.close()
    (P_, W_, (R_, lo_), C_), (dms, dcells) = max(per_bin.items(), key=lambda kv: kv[1][0])
    peak = VALU_INT16X2_TOPS if P_ == 16 else VALU_INT32_TOPS
    achieved = PATH_OPS_PER_CELL * dcells / (dms / 1e3) / 1e12
    launches = reps * chunks
    if lo_:
        # box-sweep family: <precision, lanes, column words, rows largest first (steps of 4)>
        kernel_name = "sw::sw_trace_family_kernel<%d, %d, %s, %s>" % (
            P_, W_, "true" if C_ else "false", ", ".join(str(r) for r in range(R_, lo_ - 1, -4)))
    else:
        kernel_name = "sw::sw_trace_kernel<%d, %d, %d, %s>" % (P_, W_, R_, "true" if C_ else "false")
    log("  paths: %d calls in %.3f s" % (steps, el))
    return {"value": round(fwd * steps / el / 1e9, 2), "unit": "GCUPS",
            "ms_per_call": round(el * 1e3 / steps, 3), "score_only_ms": round(score_ms, 3),
            "box_cells": int(box_cells), "record_gb": round(rec_bytes / 1e9, 3), "chunks": chunks,
            "sweep_ms": round(float(np.mean(sweep_ms)), 3), "walk_ms": round(float(np.mean(walk_ms)), 3),
            "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 2),
                         "unit": "Tops/s", "frac": round(achieved / peak, 4),
                         "traffic": stored_traffic(kernel_name, workload, cells_per_launch=dcells / launches),
                         "kernel": kernel_name, "launches": launches,
                         "launch_ms": round(dms / launches, 4),
                         "cells_per_launch": int(dcells / launches),
                         "ops_per_cell": PATH_OPS_PER_CELL,
                         "record_bytes_per_cell": 0.5}}


def roofline_only(args, batch, db, out, tuning, mode):
    """Only the roofline leg (for profiling it alone): one JSON line."""
    roof = roofline_leg(args, db, out, tuning, mode, args.workload, args.steps)
    print(json.dumps({"leg": "roofline", "config": {"workload": args.workload, "pairs": batch.n_pairs,
                                                    "routing": tuning or "built-in"},
                      "roofline": roof}), flush=True)


def serving_points(args, loads, window_s, min_requests, max_requests):
    """Open-loop serving run: a Poisson stream of requests (each 1-5,000
    pairs of the mixed draw) at each offered load (M cells/ms), submitted to
    a continuous-batching server with a device pool of args.pool_gib GiB;
    between min_requests and max_requests requests per load, about
    window_s seconds of arrivals.  Latency of a request runs from its
    scheduled arrival to its results being on the host (so a submitter that
    falls behind is charged to the request).  Returns (points, config)."""
    import queue
    import threading
    import numpy as np
    from paper_2208_12350_amd import workloads as W
    from paper_2208_12350_amd.binding import Server

    log("generating %d serving requests ..." % args.serving_requests)
    t = time.time()
    bodies = W.serving_requests(args.serving_requests)
    cells = np.array([b.cells() for b in bodies], dtype=np.float64)
    mean_cells = float(cells.mean())
    log("  mean %.3g cells per request (%.1f s)" % (mean_cells, time.time() - t))
    t = time.time()
    srv = Server(bodies[0].schemes, 0, pool_bytes=args.pool_gib << 30, slots=args.slots,
                 max_batch_pairs=args.max_batch_pairs)
    log("  server created (%.1f s)" % (time.time() - t))
    # warm-up: every slot sees a few batches before anything is timed
    for b in bodies[:4 * args.slots]:
        srv.poll(srv.submit(b), wait=True)

    points = []
    for li, load in enumerate(loads):
        lam = load * 1e6 * 1e3 / mean_cells            # requests per second
        n = int(np.clip(lam * window_s, min_requests, max_requests))
        arrivals = W.poisson_arrivals(n, lam, 2208 + li)
        which = [k % len(bodies) for k in range(n)]
        lags = [0.0] * n
        lat = [0.0] * n
        done = [0.0] * n
        handoff = queue.Queue()
        errors = []

        def collect():
            for _ in range(n):
                k, ticket = handoff.get()
                try:
                    _, ms = srv.poll(ticket, wait=True)
                except Exception as e:   # noqa: BLE001 -- reported after the run
                    errors.append(repr(e))
                    ms = float("nan")
                done[k] = time.perf_counter()
                lat[k] = ms + lags[k] * 1e3

        before = srv.stats()
        tb = srv.timing()
        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        for k in range(n):
            target = t0 + float(arrivals[k])
            while True:
                d = target - time.perf_counter()
                if d <= 0:
                    break
                time.sleep(min(d, 0.001))
            lags[k] = time.perf_counter() - target
            handoff.put((k, srv.submit(bodies[which[k]])))
        th.join()
        if errors:
            raise RuntimeError("serving requests failed: %s" % errors[:3])
        after = srv.stats()
        ta = srv.timing()
        span = max(done) - t0
        total = float(cells[which].sum())
        batches = after["batches"] - before["batches"]
        pt = {"offered_mcells_per_ms": load, "requests": n, "offered_gcups": round(load, 3),
              "sustained_gcups": round(total / span / 1e9, 2), "span_s": round(span, 3),
              "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
              "requests_per_batch": round(n / max(1, batches), 2),
              "admit_ms_per_request": round((ta["admit_ms"] - tb["admit_ms"]) / n, 3),
              "align_ms_per_batch": round((ta["align_ms"] - tb["align_ms"]) / max(1, batches), 3),
              "submit_lag_p99_ms": round(float(np.percentile(lags, 99)) * 1e3, 3)}
        log("  load %g M cells/ms: %s" % (load, pt))
        points.append(pt)
    st = srv.stats()
    srv.close()
    config = {"workload": "serving", "distinct_requests": len(bodies), "mean_cells_per_request": int(mean_cells),
              "slots": args.slots, "max_batch_pairs": args.max_batch_pairs,
              "pool_bytes": args.pool_gib << 30, "pool_peak_bytes": st["pool_peak_bytes"],
              "warmup_requests": 4 * args.slots}
    return points, config


def serving_bench(args):
    """The serving leg alone, at every load of --loads."""
    loads = [float(x) for x in args.loads.split(",")]
    points, config = serving_points(args, loads, args.window_s, 40, 500)
    top = points[-1]
    res = {
        "metric": "GCUPS, batched affine SW (score+coords), batched vs plain; p50/p99 latency",
        "value": top["sustained_gcups"], "unit": "GCUPS", "n_gpus": 1, "steps": len(points),
        "warmup": config["warmup_requests"],
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i16", "data": "synthetic",
        "config": config,
        "latency_ms": {"p50": top["p50_ms"], "p99": top["p99_ms"]},
        "serving": points,
    }
    print(json.dumps(res), flush=True)


def search_bench(args):
    """Database search (sw_search): one query against every reference of
    the search workload, inputs resident on the device, graph replay.  The
    same pairs as a plain batch (the query copied per pair) are timed beside
    it.  GCUPS = query length x total reference length per second."""
    import numpy as np
    import torch
    from paper_2208_12350_amd import workloads as W
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch
    s = W.make_search(args.workload, n_refs=args.n_pairs)
    dev = "cuda:0"
    q = torch.from_numpy(s.query).to(dev)
    r = torch.from_numpy(s.refs).to(dev)
    ro = torch.from_numpy(s.r_off).to(dev)
    out = torch.empty((s.n_refs, 5), dtype=torch.int32, device=dev)
    al = Aligner(0)
    for _ in range(args.warmup):
        al.search(q, r, ro, s.scheme, out)
    torch.cuda.synchronize()
    ts = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t = time.perf_counter()
        al.search(q, r, ro, s.scheme, out)
        ts.append((time.perf_counter() - t) * 1e3)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ref = out.clone()
    qprof_used = al.get_option("qprofile_used")
    al.close()
    cells = s.cells()
    # the same search with the forward pass on the pair table (no query profile)
    alp = Aligner(0, qprofile=0)
    alp.search(q, r, ro, s.scheme, out)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    npt = max(2, min(args.steps, 5))
    for _ in range(npt):
        alp.search(q, r, ro, s.scheme, out)
    torch.cuda.synchronize()
    elp = time.perf_counter() - tp
    alp.close()
    assert torch.equal(out, ref), "query-profile and pair-table searches differ"
    # the same pairs as a batch with the query copied per pair
    b = s.as_batch()
    db = DeviceBatch.from_host(b, dev)
    alb = Aligner(0)
    alb.align(db, out)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    nb = max(2, min(args.steps, 5))
    for _ in range(nb):
        alb.align(db, out)
    torch.cuda.synchronize()
    elb = time.perf_counter() - tb
    alb.close()
    assert torch.equal(out, ref), "search and batch results differ"
    res = {"metric": "GCUPS, database search (one query vs many references, score+coords)",
           "value": round(cells * args.steps / el / 1e9, 2), "unit": "GCUPS", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(el * 1e3 / args.steps, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i16",
           "data": "synthetic",
           "config": {"workload": args.workload, "query_len": int(s.query.size), "references": s.n_refs,
                      "cells": cells, "homologues": int(s.homolog.sum())},
           "batch_value": round(cells * nb / elb / 1e9, 2),
           "query_profile": bool(qprof_used),
           "no_profile_value": round(cells * npt / elp / 1e9, 2),
           "input_bytes": {"search": int(s.query.size + s.refs.size + 8 * s.r_off.size),
                           "batch": int(b.queries.size + b.refs.size + 8 * (b.q_off.size + b.r_off.size))},
           "latency_ms": {"p50": round(float(np.percentile(ts, 50)), 3),
                          "p99": round(float(np.percentile(ts, 99)), 3)}}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample ...")
        res["cpu_baseline"] = cpu_baseline(b)
    print(json.dumps(res), flush=True)


def calibrate_copy(dev="cuda:0"):
    """Three plain 1 GiB device-to-device copies, whose HBM byte counters
    scale those of the kernels profiled in the same process."""
    import torch
    src = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def stencil_sources_sha256():
    """Digest of the HIP source the diffusion kernels are built from."""
    import hashlib
    with open(os.path.join(ROOT, "paper_2208_12350_amd", "csrc", "sw_stencil.hip"), "rb") as f:
        return hashlib.sha256(b"sw_stencil.hip" + f.read()).hexdigest()


# the padded step's kernel on grids whose arrays exceed 512 MiB
STENCIL_KERNEL = "diffuse_padded4_kernel<16, true, true>"


def stencil_bench(args):
    """Grid diffusion (the paper's second workload, libswstencil): K steps on
    a zero-padded grid and on an unpadded grid with bounds checks, timed with
    HIP events on the launch stream.  Algorithmic traffic is 8 bytes per
    point and step (one float read, one written); the roofline is HBM."""
    import numpy as np
    import torch
    from paper_2208_12350_amd import stencil as K
    if args.calibrate_copy:
        calibrate_copy()
    sizes = [int(x) for x in args.grid.split(",")]
    steps = max(2, args.steps)
    D = 0.15
    rows = []
    for n in sizes:
        rng = torch.Generator(device="cuda").manual_seed(n)
        g = torch.rand((n, n), generator=rng, device="cuda", dtype=torch.float32)
        res = {}
        # "padded_1col": the same padded step with a pitch that is not a
        # multiple of 4, which selects the kernel with one column per lane
        for form in ("padded", "checked", "padded_1col"):
            if form.startswith("padded"):
                a = K.pad(g, K.padded_pitch(n) + (1 if form == "padded_1col" else 0))
                b = a.clone()
                step = lambda s, d: K.diffuse_padded(s, d, n, n, D)
            else:
                a, b = g.clone(), torch.empty_like(g)
                step = lambda s, d: K.diffuse_checked(s, d, D)
            for _ in range(args.warmup):
                step(a, b)
                a, b = b, a
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                step(a, b)
                a, b = b, a
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            res[form] = (ms, a[1:n + 1, 1:n + 1] if form.startswith("padded") else a)
            del b
        assert torch.equal(res["padded"][1], res["checked"][1]), "padded and checked grids differ"
        assert torch.equal(res["padded"][1], res["padded_1col"][1]), "4- and 1-column kernels differ"
        pts = n * n
        ms_p, ms_c = res["padded"][0], res["checked"][0]
        rows.append({"grid": "%dx%d" % (n, n), "step_ms_padded": round(ms_p, 4), "step_ms_checked": round(ms_c, 4),
                     "step_ms_padded_1col": round(res["padded_1col"][0], 4),
                     "gpoints_per_s_padded": round(pts / ms_p / 1e6, 2),
                     "gpoints_per_s_checked": round(pts / ms_c / 1e6, 2),
                     "padding_speedup": round(ms_c / ms_p, 3),
                     "roofline": {"bound": "hbm", "achieved": round(8 * pts / ms_p / 1e6, 1), "peak": 8000.0,
                                  "unit": "GB/s", "frac": round(8 * pts / ms_p / 1e6 / 8000.0, 4),
                                  "traffic": stored_traffic(STENCIL_KERNEL, "stencil_%d" % n, stencil_sources_sha256())}})
        del res, g
        torch.cuda.empty_cache()
    big = rows[-1]
    out = {"metric": "grid diffusion steps: Gpoints/s (padded vs bounds-checked)",
           "value": big["gpoints_per_s_padded"], "unit": "Gpoints/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": big["step_ms_padded"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "stencil", "grids": args.grid, "D": D}, "grids": rows,
           "roofline": big["roofline"]}
    if not args.no_cpu_baseline:
        from oracle import stencil as S
        n = 2500
        c = np.random.default_rng(1).random((n, n))
        t = time.perf_counter()
        k = 0
        while time.perf_counter() - t < 10.0 or k < 1:
            c = S.diffuse(c, D)
            k += 1
        dt = time.perf_counter() - t
        out["cpu_baseline"] = {"value": round(k * n * n / dt / 1e9, 4), "unit": "Gpoints/s", "cores": 1,
                               "kind": "oracle", "sample": "%d steps of the fp64 numpy oracle on a 2500x2500 grid "
                                                           "(%.1f s, one thread)" % (k, dt)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mixed")
    ap.add_argument("--secondary", default="dna_large,protein",
                    help="also measure these workloads (comma-separated; empty to skip)")
    ap.add_argument("--n-pairs", type=int, default=None, help="truncate the workload (testing only)")
    ap.add_argument("--mode", type=int, default=None, help="0 = per-bin launches, 1 = persistent")
    ap.add_argument("--streams", type=int, default=4, help="streams the persistent launches spread over")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in routing")
    ap.add_argument("--routing", default=None, help="use this routing string instead of tuning")
    ap.add_argument("--roofline-only", action="store_true", help="run only the per-launch roofline leg")
    ap.add_argument("--no-cigar", action="store_true", help="skip the alignment-path (CIGAR) leg")
    ap.add_argument("--grid", default="2500,16384", help="stencil: square grid sizes")
    ap.add_argument("--cigar-only", action="store_true", help="run only the alignment-path leg")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device to device three times (counter calibration)")
    ap.add_argument("--loads", default="1,2,5,10,20,50,100,200,500,1000,2000",
                    help="serving: offered loads in M cells/ms")
    ap.add_argument("--window-s", type=float, default=6.0, help="serving: seconds of arrivals per load")
    ap.add_argument("--serving-requests", type=int, default=300, help="serving: distinct request bodies")
    ap.add_argument("--slots", type=int, default=3, help="serving: slot workers")
    ap.add_argument("--max-batch-pairs", type=int, default=1 << 18, help="serving: pairs per merged batch")
    ap.add_argument("--pool-gib", type=int, default=16, help="serving: device pool size")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving leg of the default run (loads 1, 10 and 50 M cells/ms)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (pairs are independent, "
              "so a batch would shard by pairs across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "serving":
        serving_bench(args)
        return
    if args.workload.startswith("search_"):
        search_bench(args)
        return
    if args.workload == "stencil":
        stencil_bench(args)
        return

    res = align_leg(args, args.workload, args.steps, args.warmup, with_cigar=not args.no_cigar,
                    with_cpu=not args.no_cpu_baseline, full=True)
    if res is None:
        return
    if args.secondary:
        # the single-alphabet workloads, each measured the same way (whole
        # call, persistent + graph against plain per-bin launches, sweep
        # rooflines), without the path and CPU legs
        res["secondary"] = {}
        for name in args.secondary.split(","):
            sec = align_leg(args, name, max(5, min(args.steps, 10)), 2, with_cigar=False, with_cpu=False,
                            full=False)
            res["secondary"][name] = {k: sec[k] for k in ("value", "plain_value", "ms_per_step", "dtype")}
            res["secondary"][name]["config"] = {k: sec["config"][k] for k in ("pairs", "forward_cells",
                                                                               "reverse_cells", "routing")}
            res["secondary"][name]["roofline"] = sec["roofline"]
    if not args.no_serving and args.n_pairs is None:
        # the serving workload at its offered loads of 1, 10 and 50 M cells
        # per ms: about 12 s of Poisson arrivals each, 30 to 500 requests
        points, config = serving_points(args, [1.0, 10.0, 50.0], 12.0, 30, 500)
        res["serving"] = {"config": config, "loads": points}
    print(json.dumps(res), flush=True)


def align_leg(args, workload, steps, warmup, with_cigar, with_cpu, full):
    """Generate `workload`, tune its routing, and time whole sw_align_batch
    calls: persistent + graph (the headline) against plain per-bin launches,
    phase times, and the sweep rooflines (dominant launch, every sweep launch
    of a call, and the whole call)."""
    import numpy as np
    import torch
    from paper_2208_12350_amd import workloads as W
    from paper_2208_12350_amd.binding import Aligner, DeviceBatch

    log("generating workload %s ..." % workload)
    t = time.time()
    batch = W.make_workload(workload, n_pairs=args.n_pairs)
    log("  %d pairs, %.3g forward cells (%.1f s)" % (batch.n_pairs, batch.cells(), time.time() - t))
    dev = "cuda:0"
    db = DeviceBatch.from_host(batch, dev)
    out = torch.empty((batch.n_pairs, 5), dtype=torch.int32, device=dev)

    # routing autotuner (untimed): per-shape rates from probe launches, then
    # the routing that minimises the predicted sweep time of a sample; every
    # call is told the batch's longest query (the library then launches no
    # bin that only longer queries reach)
    tuning, tune_s = (args.routing if full else None), 0.0
    bound = "max_query=%d" % int(batch.q_len().max()) if batch.n_pairs else ""
    if full and args.calibrate_copy:
        calibrate_copy(dev)
    if tuning is None and not args.no_tune:
        from paper_2208_12350_amd import autotune as T
        log("autotuning the routing ...")
        t_tune = time.time()
        name, table, _, tile = T.tune_batch(batch, db, 0, log=log, options=bound)
        tuning = T.tuning_string(table, tile)
        tune_s = time.time() - t_tune
        log("  picked %s: %s (%.1f s)" % (name, tuning, tune_s))
    if bound and "max_query=" not in (tuning or ""):
        tuning = bound if tuning is None else tuning + ";" + bound

    def timed(al, n, warm, what):
        for k in range(warm):
            al.align(db, out)
        torch.cuda.synchronize()
        step_ms = []
        t0 = time.perf_counter()
        for k in range(n):
            ts = time.perf_counter()
            al.align(db, out)
            step_ms.append((time.perf_counter() - ts) * 1e3)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        log("  %s: %d steps in %.3f s" % (what, n, el))
        return el, step_ms

    mode = 1 if args.mode is None else args.mode
    if full and args.roofline_only:
        roofline_only(args, batch, db, out, tuning, mode)
        return None
    if full and args.cigar_only:
        al = Aligner(0, tuning)
        al.align(db, out)
        ref = out.clone()
        al.close()
        print(json.dumps({"leg": "cigar", "config": {"workload": workload, "pairs": batch.n_pairs},
                          "cigar": cigar_leg(args, db, out, ref, tuning, 0.0, workload)}), flush=True)
        return None

    # headline: persistent work-queue launch, replayed from a captured hipGraph
    al = Aligner(0, tuning, mode=mode, graph=1 if mode == 1 else 0, streams=args.streams)
    elapsed, step_ms = timed(al, steps, warmup, "mode %d" % mode)
    ref_out = out.clone()
    fwd_cells, rev_cells, i32_pairs = al.stats()
    al.close()

    # same call with HIP events around the phases (no graph replay)
    alt = Aligner(0, tuning, mode=mode, graph=0, timing=1, streams=args.streams)
    plan_ms, fwd_ms, rev_ms = [], [], []
    for k in range(max(3, min(steps, 10)) + 1):
        alt.align(db, out)
        if k:
            p, f, r = alt.timing()
            plan_ms.append(p); fwd_ms.append(f); rev_ms.append(r)
    alt.close()
    assert torch.equal(out, ref_out), "timing run disagrees with the headline run"

    roof = roofline_leg(args, db, out, tuning, mode, workload, steps)
    assert torch.equal(out, ref_out), "roofline run disagrees with the headline run"

    # plain per-bin launches on the same data
    plain = None
    if mode == 1:
        alp = Aligner(0, tuning, mode=0, graph=0)
        el_p, _ = timed(alp, max(2, min(steps, 5)), 1, "plain per-bin launches")
        alp.close()
        assert torch.equal(out, ref_out), "plain launches disagree with the persistent launch"
        plain = round(fwd_cells * max(2, min(steps, 5)) / el_p / 1e9, 2)

    ms_per_step = elapsed * 1e3 / steps
    gcups = fwd_cells * steps / elapsed / 1e9
    # the whole call (planning, both sweeps, launch gaps) against the peak
    # of the precision its cells ran at
    peak = VALU_INT16X2_TOPS if i32_pairs == 0 else VALU_INT32_TOPS
    whole = OPS_PER_CELL * (fwd_cells + rev_cells) / (ms_per_step / 1e3) / 1e12
    roof["whole_call"] = {"ms": round(ms_per_step, 3), "achieved": round(whole, 3), "frac": round(whole / peak, 4)}
    cigar = cigar_leg(args, db, out, ref_out, tuning, ms_per_step, workload) if with_cigar else None
    int16 = i32_pairs < batch.n_pairs
    res = {
        "metric": "GCUPS, batched affine SW (score+coords), batched vs plain; p50/p99 latency",
        "value": round(gcups, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i16" if int16 else "i32",
        "data": "synthetic",
        "config": {"workload": workload, "pairs": batch.n_pairs, "forward_cells": int(fwd_cells),
                   "reverse_cells": int(rev_cells), "int32_pairs": int(i32_pairs),
                   "mode": "persistent+graph" if mode == 1 else "plain per-bin launches",
                   "streams": args.streams if mode == 1 else 1,
                   "routing": tuning or "built-in", "tuning_s": round(tune_s, 2)},
        "plain_value": plain,
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 3),
                       "p99": round(float(np.percentile(step_ms, 99)), 3)},
        "phase_ms": {"plan": round(float(np.mean(plan_ms)), 3), "forward": round(float(np.mean(fwd_ms)), 3),
                     "reverse": round(float(np.mean(rev_ms)), 3)},
        "roofline": roof,
        "cigar": cigar,
    }
    if with_cpu:
        log("timing the CPU oracle on a sample ...")
        res["cpu_baseline"] = cpu_baseline(batch)
    del db, out
    torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()
