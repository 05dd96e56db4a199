#!/usr/bin/env python3
"""Throughput of the batched periodic-graph hot path on one MI355X.

One step = the whole hot path over one batch of synthetic crystals:
  cutoff multigraph build (bounds, plan, image tables, count, scan, fill)
  + KNN multigraph build (bounds, plan, image tables, ordered-stack select)
  + edge geometry forward on the cutoff edges
  + edge geometry backward to fractional coordinates and lattices, for the
    upstream gradient d loss / d length of loss = sum_e w_e exp(-(l_e - 3)^2)
    (an input of the backward pass, computed once from the lengths of this
    batch; the loss itself is the model's part and is timed separately).
The step is captured once in a HIP graph and replayed; the per-phase kernel
times come from device events in an eager run of the same step.

Default workload: 4096 structures, 1..128 atoms (log-uniform), cell lengths
2.5-20 A, angles 30-150 deg, cutoff 8 A, k = 16, one launch sequence per graph
type for the whole batch, launch parameters from the autotuner. Prints one
JSON line (see the fields below).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--config 3]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3

# algorithmic work per unit: bytes per edge / flops per candidate
BYTES_PER_EDGE_FILL = 20.0     # dst (4), image (12), length (4); src is stored by its own kernel
BYTES_PER_EDGE_SRC = 4.0       # src, written from the row offsets after the fill
BYTES_PER_EDGE_VEC = 12.0      # the edge vector, when the fill emits it
BYTES_PER_EDGE_GEOM = 36.0     # forward: read src, dst, image (20) + write vec, length (16)
BYTES_PER_EDGE_GEOM_BWD = 24.0 # backward with the length gradient only: read src, dst, image (20) + grad (4)
BYTES_PER_EDGE_KNN = 24.0      # KNN rows: src, dst, image, length
FLOPS_PER_CANDIDATE = 8.0      # 3 add + 1 mul + 2 fma (= 8 flops) per (source, destination, image)


def _parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 4])
    ap.add_argument("--no-plain", action="store_true", help="skip the per-structure launch baseline")
    ap.add_argument("--plain-structures", type=int, default=1024,
                    help="structures timed in the per-structure form (rate is per structure)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (profiler counter calibration)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch parameters")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead of a HIP graph")
    ap.add_argument("--separate-forward", action="store_true",
                    help="compute the edge vectors with the separate geometry kernel instead of taking them "
                         "from the cutoff fill")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the KNN build after the cutoff build instead of on a second stream")
    ap.add_argument("--update-loop", type=int, default=0, metavar="STEPS",
                    help="also time STEPS steps of the 64-supercell update loop (cell lists): move the "
                         "atoms, rebuild cutoff and KNN graphs, geometry forward and backward")
    ap.add_argument("--update-loop-only", action="store_true",
                    help="time only the 64-supercell update loop (STEPS from --update-loop, default 10)")
    ap.add_argument("--batch-sweep", action="store_true",
                    help="also time KNN k = 32 with ties kept on batches of 32..512 structures "
                         "(n ~ U{4..64}), with peak device memory")
    ap.add_argument("--extras-only", action="store_true",
                    help="time only the rows past the hot path on the 4096-structure batch: symmetric "
                         "closure and triplets of its KNN graph, the cutoff graph with per-atom cutoffs")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args(argv)


# The source files whose kernels make up each measured phase: hardware counters
# recorded for other versions of these files no longer describe the kernels.
PHASE_SOURCES = {
    "cutoff.count": ("sweep.hip", "mg_internal.h"),
    "cutoff.fill": ("sweep.hip", "mg_internal.h"),
    "cutoff.src": ("sweep.hip", "mg_internal.h"),
    "knn.select": ("knn.hip", "cl_tile.h", "mg_internal.h"),
    "geometry.bwd": ("geometry.hip", "mg_internal.h"),
}


def source_digest(files=None) -> str:
    """Digest of the HIP sources (all of them, or the given file names)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2307_05380_amd", "csrc")
    for name in sorted(files if files is not None else os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _counter_summary(name: str, phase: str):
    """A phase's entry of a committed hardware-counter summary, or None when the
    summary is missing or was taken on other versions of the phase's sources."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    v = t.get("phases", {}).get(phase)
    if v is None or v.get("sources_digest") != source_digest(PHASE_SOURCES.get(phase, ())):
        return None
    return v


def measured_traffic(phase: str):
    """HBM bytes per launch of a phase's kernels from the committed hardware-counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a
    device copy of known size)."""
    v = _counter_summary("hbm_traffic_4096_structures.json", phase)
    return None if v is None else v.get("bytes_per_launch")


def measured_valu(phase: str, ms: float):
    """FP32 VALU rate of a phase from the committed counter summary: the
    SQ_INSTS_VALU_FLOPS_FP32 count of its kernels (x 64 lanes) over this run's
    phase time, with the VALU issue fraction the counters gave on their run."""
    v = _counter_summary("valu_4096_structures.json", phase)
    if v is None or ms <= 0:
        return None
    tf = v["fp32_flops"] / (ms * 1e-3) / 1e12
    return {"achieved": round(tf, 3), "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / FP32_VECTOR_PEAK_TFLOPS, 4), "valu_issue_frac": v.get("valu_issue_frac"),
            "source": "SQ_INSTS_VALU_FLOPS_FP32, SQ_INSTS_VALU (rocprofv3 --pmc)"}


def _log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo), else the machine type."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def usable_cores() -> int:
    """CPUs this process may run on (its affinity set), which on a shared host
    is the share it was given, not every CPU the machine has."""
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def cpu_baseline(batch, seconds: float):
    """The FP64 oracle on a bounded sample of the batch (cutoff + KNN + geometry
    + its VJP), in a process pool over every core this process may use, plus
    the same work on one core for a smaller sample. Returns the dict for the
    JSON line."""
    import numpy as np

    import oracle

    cores = usable_cores()
    # size the sample from a quick single-structure timing
    def run(structs, procs):
        t0 = time.perf_counter()
        g = oracle.cutoff_graph64(batch.lattices, batch.frac, batch.batch_ptr, batch.cutoff,
                                  structures=structs, processes=procs)
        oracle.knn_graph64(batch.lattices, batch.frac, batch.batch_ptr, batch.k, structures=structs,
                           processes=procs)
        v, ln = oracle.edge_geometry64(batch.lattices, batch.frac, batch.batch_ptr, g.src, g.dst, g.image)
        oracle.edge_geometry_vjp64(batch.lattices, batch.frac, batch.batch_ptr, g.src, g.dst, g.image,
                                   None, np.ones_like(ln))
        return time.perf_counter() - t0, g.num_edges

    probe = list(range(0, batch.B, max(1, batch.B // 64)))[:64]
    dt, _ = run(probe, cores)
    per = dt / len(probe)
    S = int(min(batch.B, max(len(probe), seconds / max(per, 1e-6))))
    rng = np.random.default_rng(0)
    sample = sorted(rng.choice(batch.B, S, replace=False).tolist()) if S < batch.B else list(range(batch.B))
    dt, E = run(sample, cores)
    # one core: a smaller sample of the same draw, about a quarter of the time budget
    S1 = int(min(len(sample), max(8, 0.25 * seconds * len(sample) / max(dt * cores, 1e-6))))
    sample1 = sample[::max(1, len(sample) // S1)][:S1]
    dt1, E1 = run(sample1, 1)
    return {"value": len(sample) / dt, "unit": "structures/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sample)} of {batch.B} structures drawn uniformly (seed 0), FP64 numpy "
                      f"cutoff+KNN+geometry+VJP, {E} cutoff edges, {dt:.1f} s wall on {cores} processes",
            "cpu": cpu_model(), "cpu_count_os": os.cpu_count(),
            "single_core": {"value": round(len(sample1) / dt1, 3), "unit": "structures/s",
                            "sample": f"every {max(1, len(sample) // S1)}-th of the sample above, "
                                      f"{len(sample1)} structures, {E1} cutoff edges, {dt1:.1f} s wall"}}


def main(argv=None):
    args = _parse(argv)
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the batch shards over GPUs "
                                   "by structure with no communication (see DESIGN.md), and no "
                                   "multi-GPU figure is produced", "n_gpus": args.gpus}))
        return 2
    import numpy as np
    import torch

    from paper_2307_05380_amd import _lib, graph, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.update_loop_only:
        res = update_loop(dev, args.update_loop or 10, cpu_sample=not args.no_cpu_baseline, tune_first=not args.no_tune)
        print(json.dumps({"update_loop": res, "source_digest": source_digest()}))
        return 0
    if args.extras_only:
        print(json.dumps({"extras": extras(dev), "source_digest": source_digest()}))
        return 0
    batch = inputs.make_config(args.config)
    B, N, k, c = batch.B, batch.N, batch.k, batch.cutoff
    L = torch.from_numpy(batch.lattices).to(dev)
    X = torch.from_numpy(batch.frac).to(dev)
    P = torch.from_numpy(batch.batch_ptr).to(dev)
    _log(args, f"workload config{args.config}: B={B} N={N} cutoff={c} k={k}")

    # cell lists only pay off for structures of >= 512 atoms
    opts = _lib.MG_OPT_CELL_LIST_OFF if int(batch.counts().max()) < graph.CL_MIN_ATOMS else 0
    tuning = None
    if not args.no_tune:
        from paper_2307_05380_amd import tune
        best = tune.autotune(L, X, P, c, k, use_cache=False)
        tuning = {**best["cutoff"], **best["knn"]}
        _log(args, "tuning", tuning, best["ms"])
    # ---- sizing (untimed): exact edge count and image-table sizes
    g0 = graph.cutoff_graph(L, X, P, c, opts=opts)
    E = g0.num_edges
    cut_images = g0.report.images_needed
    k0 = graph.knn_graph(L, X, P, k, opts=opts)
    knn_images = k0.report.images_needed
    del g0, k0
    # the edge vectors and lengths come out of the cutoff fill (fused), or from
    # the separate geometry kernel
    fused = not args.separate_forward
    cb = graph.CutoffBuilder(B, N, E, cut_images, dev, vec=fused)
    kb = graph.KnnBuilder(B, N, k, knn_images, dev)
    geo = graph.GeometryRunner(B, N, dev)
    if fused:
        vec, length = cb.vec, cb.length
    else:
        vec = torch.empty((E, 3), dtype=torch.float32, device=dev)
        length = torch.empty(E, dtype=torch.float32, device=dev)
    gf = torch.empty_like(X)
    gL = torch.empty_like(L)
    ne = cb.rep[:1]     # device edge count written by the cutoff call

    # upstream gradient of the loss at this batch (the model's part, untimed)
    cb.run(L, X, P, c, opts)
    if not fused:
        geo.forward(L, X, P, cb.src, cb.dst, cb.image, vec, length, num_edges=ne)
    w = torch.from_numpy(inputs.loss_weights(E)).to(dev)

    def loss_grad():
        u = length - 3.0
        return -2.0 * w * u * torch.exp(-u * u)

    glen = loss_grad()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        loss_grad()
    torch.cuda.synchronize()
    ms_loss = (time.perf_counter() - t0) * 1e3 / 5

    def step():
        cb.run(L, X, P, c, opts)
        kb.run(L, X, P, opts)
        if not fused:
            geo.forward(L, X, P, cb.src, cb.dst, cb.image, vec, length, num_edges=ne)
        geo.backward(L, X, P, cb.src, cb.dst, cb.image, None, glen, gf, gL, num_edges=ne)

    # ---- eager run with per-phase device events
    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    rep_c = cb.report()
    rep_k = kb.report()
    assert rep_c.num_edges == E and not (rep_c.flags & ~_lib.MG_FLAG_KNN_EXTENDED), rep_c
    # a KNN source with a RANGE / IMAGES / ... flag gets invalid rows: none may be timed
    assert not (rep_k.flags & ~_lib.MG_FLAG_KNN_EXTENDED), rep_k
    ref = [t.clone() for t in (cb.src, cb.dst, cb.image, kb.dst, kb.image, length, gf, gL)]
    _lib.profile_enable(True)
    _lib.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
    _lib.profile_enable(False)
    phases = _lib.profile_read()

    # The KNN build does not depend on the cutoff build or on the geometry, so the
    # timed step runs it on a second stream (default priority) that forks from and
    # joins the main one; its work overlaps the cutoff sweeps and the geometry.
    knn_stream = None if args.no_overlap else torch.cuda.Stream()

    # The KNN build forks either at the start of the step (it then shares the
    # GPU with the cutoff count, which is VALU-bound like itself) or after the
    # cutoff build (it then shares it with the geometry backward, which is
    # bound by memory); the joint tuning below picks the faster schedule.
    schedule = {"knn_fork": "start"}

    def step_overlap():
        main = torch.cuda.current_stream()
        after = schedule["knn_fork"] == "after_cutoff"
        if not after:
            knn_stream.wait_stream(main)
            with torch.cuda.stream(knn_stream):
                kb.run(L, X, P, opts)
        cb.run(L, X, P, c, opts)
        if after:
            knn_stream.wait_stream(main)
            with torch.cuda.stream(knn_stream):
                kb.run(L, X, P, opts)
        if not fused:
            geo.forward(L, X, P, cb.src, cb.dst, cb.image, vec, length, num_edges=ne)
        geo.backward(L, X, P, cb.src, cb.dst, cb.image, None, glen, gf, gL, num_edges=ne)
        main.wait_stream(knn_stream)

    # ---- the timed region: K replays of the captured step (or K eager steps)
    step_timed = step if args.no_overlap else step_overlap

    def capture(fn):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fn()
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        return g

    if tuning is not None and not args.no_overlap and not args.no_graph:
        # The two streams share the GPU, so the launch shapes that are best for
        # each build alone are not best together: time the captured step for a
        # few grid sizes of both sweeps (the KNN search radius stays as tuned).
        best_ms, best_cfg = None, None
        for fork in ("start", "after_cutoff"):
            schedule["knn_fork"] = fork
            for cw in (16, 32, 64):
                for kw in (1, 2, 4, 16):
                    cfg = {**tuning, "cutoff_wgs_per_cu": cw, "knn_wgs_per_cu": kw}
                    _lib.set_tuning(**cfg)
                    g = capture(step_timed)
                    for _ in range(3):
                        g.replay()
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(10):
                        g.replay()
                    e1.record()
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / 10
                    del g
                    if best_ms is None or ms < best_ms:
                        best_ms, best_cfg = ms, (cfg, fork)
        tuning, schedule["knn_fork"] = best_cfg
        _lib.set_tuning(**tuning)
        _log(args, "overlap tuning", tuning, schedule, round(best_ms, 4))
    run = step_timed
    if not args.no_graph:
        cg = capture(step_timed)
        run = cg.replay
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        run()
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / max(args.steps, 1)
    ms_step_ev = ev0.elapsed_time(ev1) / max(args.steps, 1)
    # the replayed step reproduces the eager one (graph edges exactly, gradients to rounding)
    out_now = [cb.src, cb.dst, cb.image, kb.dst, kb.image, length, gf, gL]
    for a, r in zip(out_now[:6], ref[:6]):
        assert torch.equal(a, r), "graph replay differs from the eager step"
    for a, r in zip(out_now[6:], ref[6:]):
        assert float((a - r).abs().max()) <= 1e-4 * max(float(r.abs().max()), 1e-30)

    # ---- roofline of every phase; the dominant one goes into "roofline"
    per = {}
    work = {
        "cutoff.fill": ("hbm", (BYTES_PER_EDGE_FILL + (BYTES_PER_EDGE_VEC if fused else 0.0)) * E),
        "cutoff.src": ("hbm", BYTES_PER_EDGE_SRC * E),
        "cutoff.count": ("alu", FLOPS_PER_CANDIDATE * rep_c.candidates),
        "knn.select": ("alu", FLOPS_PER_CANDIDATE * rep_k.candidates),
        "geometry.fwd": ("hbm", BYTES_PER_EDGE_GEOM * E),
        "geometry.bwd": ("hbm", BYTES_PER_EDGE_GEOM_BWD * E),
    }
    for name, (ms, cnt) in phases.items():
        avg = ms / max(cnt, 1)
        d = {"ms_avg": round(avg, 5), "launches": cnt}
        if name in work:
            bound, amount = work[name]
            if bound == "hbm":
                ach = amount / (avg * 1e-3) / 1e9
                d.update(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                         frac=round(ach / HBM_PEAK_GBS, 4))
            else:
                ach = amount / (avg * 1e-3) / 1e12
                d.update(bound="alu", achieved=round(ach, 3), peak=FP32_VECTOR_PEAK_TFLOPS, unit="TFLOP/s",
                         frac=round(ach / FP32_VECTOR_PEAK_TFLOPS, 4))
            # executed FP32 work from the hardware counters, beside the algorithmic rate
            cv = measured_valu(name, avg)
            if cv is not None:
                d["valu_counters"] = cv
        per[name] = d
    dom = max((n for n in per if n in work), key=lambda n: per[n]["ms_avg"], default=None)
    roof = None
    if dom:
        d = per[dom]
        roof = {"kernel": dom, "bound": d["bound"], "achieved": d["achieved"], "peak": d["peak"],
                "unit": d["unit"], "frac": d["frac"], "traffic": measured_traffic(dom)}

    # ---- the whole step against the same roof: the algorithmic bytes of all its
    # HBM-bound phases (cutoff rows with vectors, src, KNN rows, backward) over the
    # measured time of the step
    step_bytes = ((BYTES_PER_EDGE_FILL + BYTES_PER_EDGE_SRC + BYTES_PER_EDGE_GEOM_BWD
                   + (BYTES_PER_EDGE_VEC if fused else BYTES_PER_EDGE_GEOM)) * E + BYTES_PER_EDGE_KNN * N * k)
    step_ach = step_bytes / (ms_step * 1e-3) / 1e9
    roof_step = {"bound": "hbm", "algorithmic_bytes": int(step_bytes), "achieved": round(step_ach, 1),
                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(step_ach / HBM_PEAK_GBS, 4)}

    # ---- per-structure launch form (the plain method, one launch sequence per structure)
    plain = None
    if not args.no_plain:
        plain = plain_form(args, batch, L, X, P, cb, dev, fused)

    out = {
        "metric": "structures/s & edges/s, batched cutoff+KNN build fwd+bwd vs plain; % roofline",
        "value": round(B / (ms_step / 1e3), 1),
        "unit": "structures/s",
        "edges_per_s": round((E + N * k) / (ms_step / 1e3), 1),
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4), "ms_per_step_events": round(ms_step_ev, 4),
        "ms_per_step_eager": round(ms_eager, 4), "timed": "eager" if args.no_graph else "hip_graph",
        "ms_loss_model_part": round(ms_loss, 4), "tuning": tuning,
        "schedule": None if args.no_overlap else dict(schedule), "source_digest": source_digest(),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{B} structures, {N} atoms, cutoff {c} A, k {k}, one batched launch sequence "
                               "per graph type" + ("" if args.no_graph else ", captured in a HIP graph")
                               + ("" if args.no_overlap else "; the KNN build on a second stream")
                               + ("; edge vectors and lengths emitted by the cutoff fill" if fused
                                  else "; edge vectors and lengths by the separate geometry kernel"),
                   "structures": B, "atoms": N, "cutoff_edges": E, "knn_edges": N * k, "cutoff": c, "k": k},
        "roofline": roof,
        "roofline_step": roof_step,
        "phases": per,
        "plain": plain,
        "vs_plain": round((B / (ms_step / 1e3)) / plain["value"], 2) if plain else None,
        "report": {"cutoff_candidates": rep_c.candidates, "cutoff_images": rep_c.images_needed,
                   "knn_candidates": rep_k.candidates, "knn_images": rep_k.images_needed,
                   "knn_extended_sources": rep_k.knn_extended, "cutoff_flags": rep_c.flags,
                   "knn_flags": rep_k.flags},
    }
    if args.copy_calibration_mb > 0:
        n = args.copy_calibration_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        bb = torch.empty_like(a)
        bb.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = n * 4
    if args.batch_sweep:
        out["batch_sweep"] = batch_sweep(dev)
    if args.update_loop > 0:
        out["update_loop"] = update_loop(dev, args.update_loop, tune_first=not args.no_tune)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(batch, args.cpu_seconds)
        out["cpu_baseline"]["value"] = round(out["cpu_baseline"]["value"], 2)
    print(json.dumps(out))
    return 0


def update_loop(dev, steps: int, warmup: int = 2, cpu_sample: bool = False, tune_first: bool = True):
    """64 supercells (8-atom base cells tiled 8..16 times per direction, ~10^6
    atoms): every step adds a Cartesian N(0, 0.02 A) move to every atom, then
    rebuilds the cutoff graph (5 A, edge vectors and lengths from its fill) and
    the KNN graph (k = 32), both through cell lists, and runs the edge geometry
    backward (a fixed random upstream gradient on the lengths). Moves are drawn
    beforehand; the timed region holds the coordinate update and the three
    library calls."""
    import numpy as np
    import torch

    from paper_2307_05380_amd import _lib, graph, inputs

    b = inputs.make_config5()
    L = torch.from_numpy(b.lattices).to(dev)
    X = torch.from_numpy(b.frac).to(dev)
    P = torch.from_numpy(b.batch_ptr).to(dev)
    tuning = None
    if tune_first:   # launch shapes and the cell-list KNN threshold for this workload
        from paper_2307_05380_amd import tune
        best = tune.autotune(L, X, P, b.cutoff, b.k, use_cache=False)
        tuning = {**best["cutoff"], **best["knn"]}
    n_steps = warmup + steps
    deltas = torch.from_numpy(np.stack([inputs.config5_step_delta(b, s) for s in range(n_steps)])).to(dev)
    g0 = graph.cutoff_graph(L, X, P, b.cutoff)
    cap = int(g0.num_edges * 1.15) + 4096
    del g0
    cb = graph.CutoffBuilder(b.B, b.N, cap, 4096, dev, vec=True)
    kb = graph.KnnBuilder(b.B, b.N, b.k, 4096, dev)
    geo = graph.GeometryRunner(b.B, b.N, dev)
    gf = torch.empty_like(X)
    gL = torch.empty_like(L)
    glen = torch.from_numpy(np.random.default_rng(5).normal(size=cap).astype(np.float32)).to(dev)
    ne = cb.rep[:1]
    hist = torch.zeros(n_steps, dtype=torch.int64, device=dev)
    flags = torch.zeros(n_steps, dtype=torch.int64, device=dev)

    def step(s):
        X.add_(deltas[s])
        cb.run(L, X, P, b.cutoff, 0)
        kb.run(L, X, P, 0)
        geo.backward(L, X, P, cb.src, cb.dst, cb.image, None, glen, gf, gL, num_edges=ne)
        hist[s] = cb.rep[0]
        flags[s] = cb.rep[4] | kb.rep[4]

    for s in range(warmup):
        step(s)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for s in range(warmup, n_steps):
        step(s)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    h = hist.cpu().numpy()[warmup:]
    f = int(np.bitwise_or.reduce(flags.cpu().numpy() & 0xFFFFFFFF))
    bad = f & ~_lib.MG_FLAG_KNN_EXTENDED
    assert not bad, f"update loop flags 0x{f:x}"
    E = float(h.mean())
    out = {"supercells": b.B, "atoms": b.N, "steps": steps, "ms_per_step": round(ms, 4),
           "cutoff_edges_mean": int(E), "knn_edges": b.N * b.k, "cutoff": b.cutoff, "k": b.k,
           "edges_per_s": round((E + b.N * b.k) / (ms / 1e3), 1),
           "structures_per_s": round(b.B / (ms / 1e3), 1), "tuning": tuning}
    if cpu_sample:
        out["cpu_oracle_extrapolated"] = update_loop_cpu(b)
    return out


def update_loop_cpu(b, sources: int = 24):
    """The FP64 oracle on a few sources of one supercell (cutoff against every
    atom and image, KNN, geometry and its VJP on those sources' edges), on one
    core, extrapolated per atom to a whole update step of the 64 supercells.
    A whole step cannot be brute-forced (a 32768-atom supercell alone has about
    2.9e10 candidates); the figure is labelled extrapolated."""
    import numpy as np

    import oracle

    q = int(np.argmax(np.diff(b.batch_ptr)))   # the largest supercell: the per-source cost grows with n
    L, x = b.structure(q)
    n = x.shape[0]
    srcs = sorted(np.random.default_rng(0).choice(n, sources, replace=False).tolist())
    t0 = time.perf_counter()
    s, d, t, ln = oracle.cutoff_sources64(L, x, b.cutoff, srcs)
    oracle.knn_structure64(L, x, b.k, sources=srcs)
    ptr = np.array([0, n], np.int64)
    v, l64 = oracle.edge_geometry64(L[None], x, ptr, s, d, t)
    oracle.edge_geometry_vjp64(L[None], x, ptr, s, d, t, None, np.ones_like(l64))
    dt = time.perf_counter() - t0
    per_atom = dt / len(srcs)
    # the per-source cost is about linear in the supercell's atom count
    step_s = per_atom * float((np.diff(b.batch_ptr).astype(np.float64) ** 2).sum()) / n
    return {"value": round(b.B / step_s, 6), "unit": "structures/s", "cores": 1, "kind": "oracle",
            "extrapolated": True,
            "sample": f"{len(srcs)} sources of the {n}-atom supercell, {dt:.1f} s; per-source time scaled "
                      f"by n_s / {n} for every supercell s (the oracle compares a source with all n_s atoms)",
            "seconds_per_step": round(step_s, 1)}


def _time_calls(call, reps: int = 20) -> float:
    """Milliseconds per call of `call` (device events around `reps` calls, after one)."""
    import torch

    call()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        call()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _hbm(ms: float, nbytes: float) -> dict:
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"ms": round(ms, 4), "algorithmic_bytes": int(nbytes), "achieved": round(gbs, 1), "peak": 8000.0,
            "unit": "GB/s", "frac": round(gbs / 8000.0, 4)}


def extras(dev, reps: int = 20):
    """The rows past the hot path on the 4096-structure batch (cutoff 8 A, k = 16),
    one library call per timing with preallocated buffers (device events):
    symmetric closure of the KNN graph (read dst, image, length = 20 B per input
    edge; write src, dst, image, length = 24 B per output edge), triplets with
    angles of the KNN graph (12 B per triplet written, the edge vectors read
    once), and the cutoff graph with per-atom cutoffs c_i ~ U(6, 8) A (seeded)
    against the same call at one cutoff of 8 A (dst, image, length and src: 24 B
    per edge)."""
    import numpy as np
    import torch

    from paper_2307_05380_amd import _lib, graph, inputs
    from paper_2307_05380_amd.graph import _ptr, _stream

    lib = _lib.load()
    b = inputs.make_config3()
    L = torch.from_numpy(b.lattices).to(dev)
    X = torch.from_numpy(b.frac).to(dev)
    P = torch.from_numpy(b.batch_ptr).to(dev)
    N, k = b.N, b.k
    opts = _lib.MG_OPT_CELL_LIST_OFF
    out = {}
    g = graph.knn_graph(L, X, P, k, opts=opts)
    E = N * k
    row_ptr = torch.arange(0, E + 1, k, dtype=torch.int64, device=dev)
    dst, image, length = g.dst.contiguous(), g.image.contiguous(), g.length.contiguous()
    rep = torch.zeros(_lib.REPORT_BYTES // 8, dtype=torch.int64, device=dev)

    # symmetric closure (f1)
    cap = 2 * E
    ws = torch.empty(max(int(lib.mg_symmetrize_workspace_bytes(N, E)), 256), dtype=torch.uint8, device=dev)
    so = [torch.empty(cap, dtype=torch.int32, device=dev), torch.empty(cap, dtype=torch.int32, device=dev),
          torch.empty((cap, 3), dtype=torch.int32, device=dev), torch.empty(cap, dtype=torch.float32, device=dev)]
    optr = torch.empty(N + 1, dtype=torch.int64, device=dev)

    def sym():
        _lib.check(lib.mg_symmetrize(_ptr(row_ptr), N, _ptr(dst), _ptr(image), _ptr(length), E, cap,
                                     *[_ptr(o) for o in so], _ptr(optr), _ptr(rep), _ptr(ws), ws.numel(),
                                     _stream(dev)), lib)

    ms = _time_calls(sym, reps)
    S = graph.Report.from_tensor(rep).num_edges
    out["symmetrize"] = {"input_edges": E, "output_edges": S,
                         **_hbm(ms, 20.0 * E + 24.0 * S + 16.0 * (N + 1))}
    del ws, so, optr

    # triplets with angles (f2)
    geo = graph.GeometryRunner(b.B, N, dev)
    vec = torch.empty((E, 3), dtype=torch.float32, device=dev)
    lv = torch.empty(E, dtype=torch.float32, device=dev)
    geo.forward(L, X, P, g.src, dst, image, vec, lv)
    T = N * k * (k - 1)
    ws = torch.empty(max(int(lib.mg_triplets_workspace_bytes(N)), 256), dtype=torch.uint8, device=dev)
    to = [torch.empty(T, dtype=torch.int32, device=dev), torch.empty(T, dtype=torch.int32, device=dev),
          torch.empty(T, dtype=torch.float32, device=dev)]
    tptr = torch.empty(N + 1, dtype=torch.int64, device=dev)

    def trip():
        _lib.check(lib.mg_triplets(_ptr(row_ptr), N, E, _ptr(vec), T, *[_ptr(o) for o in to], _ptr(tptr),
                                   _ptr(rep), _ptr(ws), ws.numel(), _stream(dev)), lib)

    ms = _time_calls(trip, reps)
    got = graph.Report.from_tensor(rep).num_edges
    out["triplets"] = {"edges": E, "triplets": got, **_hbm(ms, 12.0 * got + 12.0 * E + 16.0 * (N + 1))}
    del ws, to, tptr, vec, lv, g

    # per-atom cutoffs (f3) against one cutoff
    radii = torch.from_numpy(np.random.default_rng(230705380 + 60).uniform(6.0, 8.0, N).astype(np.float32)).to(dev)
    gr = graph.cutoff_graph(L, X, P, radii, opts=opts)
    Er, icap = gr.num_edges, gr.report.images_needed
    del gr
    cb = graph.CutoffBuilder(b.B, N, Er, icap, dev)
    ms_r = _time_calls(lambda: cb.run(L, X, P, radii, opts), reps)
    assert cb.report().num_edges == Er
    g8 = graph.cutoff_graph(L, X, P, 8.0, opts=opts)
    E8, icap8 = g8.num_edges, g8.report.images_needed
    del g8, cb
    cb = graph.CutoffBuilder(b.B, N, E8, icap8, dev)
    ms_8 = _time_calls(lambda: cb.run(L, X, P, 8.0, opts), reps)
    out["per_atom_cutoffs"] = {"edges": Er, "edges_per_s": round(Er / (ms_r * 1e-3), 1), **_hbm(ms_r, 24.0 * Er),
                               "one_cutoff_8A": {"edges": E8, "edges_per_s": round(E8 / (ms_8 * 1e-3), 1),
                                                 **_hbm(ms_8, 24.0 * E8)}}
    return out


def batch_sweep(dev, sizes=(32, 64, 128, 256, 512), k=32, reps=10):
    """KNN graph with ties kept (the paper's selection d <= d_k) at k = 32 for
    batches of 32..512 structures drawn like the 256-structure batch (n ~ U{4..64},
    lengths 3-15 A, angles 60-120 deg): milliseconds per batch (device events,
    one library call per batch, buffers preallocated) and the peak device memory
    of a call (outputs + workspace), per batch size."""
    import torch

    from paper_2307_05380_amd import _lib, graph, inputs
    from paper_2307_05380_amd.graph import _ptr, _stream

    res = []
    lib = _lib.load()
    for B in sizes:
        b = inputs.make_config2(B=B)
        L = torch.from_numpy(b.lattices).to(dev)
        X = torch.from_numpy(b.frac).to(dev)
        P = torch.from_numpy(b.batch_ptr).to(dev)
        g = graph.knn_graph_ties(L, X, P, k, opts=_lib.MG_OPT_CELL_LIST_OFF)     # sizes
        cap, icap = max(g.report.num_edges, 1), max(g.report.images_needed, 1)
        del g
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats(dev)
        base = torch.cuda.memory_allocated(dev)
        ws = torch.empty(int(lib.mg_knn_ties_workspace_bytes(B, b.N, k, icap)), dtype=torch.uint8, device=dev)
        outs = [torch.empty(cap, dtype=torch.int32, device=dev), torch.empty(cap, dtype=torch.int32, device=dev),
                torch.empty((cap, 3), dtype=torch.int32, device=dev), torch.empty(cap, device=dev)]
        row_ptr = torch.empty(b.N + 1, dtype=torch.int64, device=dev)
        rep = torch.zeros(_lib.REPORT_BYTES // 8, dtype=torch.int64, device=dev)

        def call():
            _lib.check(lib.mg_knn_graph_ties(_ptr(L), _ptr(X), _ptr(P), B, b.N, k, cap, *[_ptr(o) for o in outs],
                                             _ptr(row_ptr), _ptr(rep), _ptr(ws), ws.numel(),
                                             _lib.MG_OPT_CELL_LIST_OFF, _stream(dev)), lib)

        call()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            call()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        peak = torch.cuda.max_memory_allocated(dev) - base
        r = graph.Report.from_tensor(rep)
        res.append({"structures": B, "atoms": b.N, "edges": r.num_edges, "ms_per_batch": round(ms, 4),
                    "structures_per_s": round(B / (ms / 1e3), 1), "peak_mb": round(peak / 2 ** 20, 2)})
        del ws, outs
    return res


def plain_form(args, batch, L, X, P, cb, dev, fused=True):
    """The same kernels launched once per structure: every structure gets its own
    cutoff call (with the edge vectors when `fused`, else followed by the
    geometry forward), KNN call and geometry backward. Times the first
    `plain_structures` structures."""
    import numpy as np
    import torch

    from paper_2307_05380_amd import _lib, graph

    S = min(args.plain_structures, batch.B)
    ptr = batch.batch_ptr
    row = cb.row_ptr.cpu().numpy()
    k = batch.k
    nmax = int(np.diff(ptr).max())
    local_ptr = torch.tensor([[0, int(ptr[s + 1] - ptr[s])] for s in range(S)], dtype=torch.int64, device=dev)
    cap_max = int(max(row[ptr[s + 1]] - row[ptr[s]] for s in range(S)))
    cbs = graph.CutoffBuilder(1, nmax, max(cap_max, 1), 1 << 16, dev, vec=fused)
    kbs = graph.KnnBuilder(1, nmax, k, 1 << 16, dev)
    geo = graph.GeometryRunner(1, nmax, dev)
    vec = torch.empty((max(cap_max, 1), 3), device=dev)
    ln = torch.empty(max(cap_max, 1), device=dev)
    gf = torch.empty((nmax, 3), device=dev)
    gL = torch.empty((1, 3, 3), device=dev)
    glen = torch.ones(max(cap_max, 1), device=dev)
    lib = cbs.lib
    from paper_2307_05380_amd.graph import _ptr, _stream
    import ctypes

    def one(s):
        a0, a1 = int(ptr[s]), int(ptr[s + 1])
        n = a1 - a0
        Ls = L[s:s + 1]
        Xs = X[a0:a1]
        ps = local_ptr[s]
        cbs.N = n
        kbs.N = n
        cbs.run(Ls, Xs, ps, batch.cutoff, _lib.MG_OPT_CELL_LIST_OFF)
        kbs.run(Ls, Xs, ps, _lib.MG_OPT_CELL_LIST_OFF)
        e = int(row[a1] - row[a0])
        if e:
            geo.N = n
            if not fused:
                geo.forward(Ls, Xs, ps, cbs.src[:e], cbs.dst[:e], cbs.image[:e], vec, ln)
            geo.backward(Ls, Xs, ps, cbs.src[:e], cbs.dst[:e], cbs.image[:e], None, glen, gf, gL)

    for s in range(min(8, S)):
        one(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(S):
        one(s)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"value": round(S / dt, 1), "unit": "structures/s", "structures": S,
            "form": "one launch sequence per structure (same kernels), first S structures of the batch"}


if __name__ == "__main__":
    sys.exit(main())
