"""Autotuner for the launch parameters of the graph sweeps.

Tunables (``mg_tuning`` in include/matgraph.h):
- cutoff_wgs_per_cu: persistent workgroups per CU of the cutoff count/fill sweeps;
- cutoff_slots:      destination atoms per lane per image step for structures
                     with more than 64 atoms (1, 2 or 4);
- knn_wgs_per_cu:    persistent workgroups per CU of the KNN sweep;
- knn_lambda_x4:     4x the expected number of candidates per neighbour that
                     the first KNN search radius is sized for.

Every candidate is timed with device events over repeated calls and must give
bit-identical edges to the first candidate; the fastest is kept. Results are
cached as JSON keyed by GPU architecture and workload signature
(``MG_TUNE_CACHE`` or ``~/.cache/matgraph/tune.json``).
"""
from __future__ import annotations

import itertools
import json
import os

import torch

from . import _lib, graph

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "matgraph", "tune.json")

CUTOFF_SPACE = {"cutoff_wgs_per_cu": [2, 4, 8, 16], "cutoff_slots": [1, 2, 4]}
KNN_SPACE = {"knn_wgs_per_cu": [2, 4, 8, 16], "knn_lambda_x4": [4, 6, 8, 12]}


def _arch(device) -> str:
    p = torch.cuda.get_device_properties(device)
    return getattr(p, "gcnArchName", p.name)


def signature(B: int, N: int, cutoff: float, k: int) -> str:
    """Workload key: batch size and mean atoms per structure in coarse buckets."""
    nb = 1 << max(0, int(B).bit_length() - 1)
    mean = N / max(B, 1)
    mb = 1 << max(0, int(mean).bit_length() - 1)
    return f"B{nb}-n{mb}-c{round(float(cutoff))}-k{int(k)}"


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def _snapshot(builder, count):
    return [t[:count].clone() for t in (builder.src, builder.dst, builder.image, builder.length)]


def _same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


def tune(lattices, frac, batch_ptr, cutoff: float, k: int, reps: int = 5, space_cutoff=None,
         space_knn=None, verbose: bool = False) -> dict:
    """Time every candidate on this batch; returns {"cutoff": {...}, "knn": {...}, "ms": {...}}."""
    B, N = int(lattices.shape[0]), int(frac.shape[0])
    dev = frac.device
    base = _lib.get_tuning()
    g = graph.cutoff_graph(lattices, frac, batch_ptr, cutoff)
    E, icap = g.num_edges, g.report.images_needed
    kg = graph.knn_graph(lattices, frac, batch_ptr, k)
    kcap = kg.report.images_needed
    cb = graph.CutoffBuilder(B, N, max(E, 1), max(icap, 1), dev)
    kb = graph.KnnBuilder(B, N, k, max(kcap, 1), dev)
    results = {"cutoff": [], "knn": []}
    ref = None
    space_cutoff = space_cutoff or CUTOFF_SPACE
    for vals in itertools.product(*space_cutoff.values()):
        cfg = dict(zip(space_cutoff.keys(), vals))
        _lib.set_tuning(**cfg)
        ms = _time(lambda: cb.run(lattices, frac, batch_ptr, cutoff), reps)
        snap = _snapshot(cb, E)
        if ref is None:
            ref = snap
        ok = _same(ref, snap)
        results["cutoff"].append((ms, cfg, ok))
        if verbose:
            print("cutoff", cfg, f"{ms:.4f} ms", "ok" if ok else "MISMATCH", flush=True)
    ref = None
    space_knn = space_knn or KNN_SPACE
    for vals in itertools.product(*space_knn.values()):
        cfg = dict(zip(space_knn.keys(), vals))
        _lib.set_tuning(**cfg)
        ms = _time(lambda: kb.run(lattices, frac, batch_ptr), reps)
        snap = _snapshot(kb, N * k)
        if ref is None:
            ref = snap
        ok = _same(ref, snap)
        results["knn"].append((ms, cfg, ok))
        if verbose:
            print("knn", cfg, f"{ms:.4f} ms", "ok" if ok else "MISMATCH", flush=True)
    _lib.set_tuning(**base)
    bad = [c for _, c, ok in results["cutoff"] + results["knn"] if not ok]
    if bad:
        raise RuntimeError(f"tuning candidates changed the graph: {bad}")
    best_c = min(results["cutoff"], key=lambda r: r[0])
    best_k = min(results["knn"], key=lambda r: r[0])
    return {"cutoff": best_c[1], "knn": best_k[1], "ms": {"cutoff": best_c[0], "knn": best_k[0]},
            "all": {"cutoff": [(m, c) for m, c, _ in results["cutoff"]],
                    "knn": [(m, c) for m, c, _ in results["knn"]]}}


def cache_path() -> str:
    return os.environ.get("MG_TUNE_CACHE", DEFAULT_CACHE)


def load(device, sig: str) -> dict | None:
    try:
        with open(cache_path()) as f:
            return json.load(f).get(_arch(device), {}).get(sig)
    except (OSError, ValueError):
        return None


def store(device, sig: str, best: dict):
    path = cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    data.setdefault(_arch(device), {})[sig] = {"cutoff": best["cutoff"], "knn": best["knn"], "ms": best["ms"]}
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    with open(path + ".tmp", "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(path + ".tmp", path)


def apply(best: dict):
    _lib.set_tuning(**best["cutoff"], **best["knn"])


def autotune(lattices, frac, batch_ptr, cutoff: float, k: int, reps: int = 5, use_cache: bool = True,
             verbose: bool = False) -> dict:
    """Load the cached best parameters for this workload or tune and cache them; applies them."""
    B, N = int(lattices.shape[0]), int(frac.shape[0])
    sig = signature(B, N, cutoff, k)
    best = load(frac.device, sig) if use_cache else None
    if best is None:
        best = tune(lattices, frac, batch_ptr, cutoff, k, reps=reps, verbose=verbose)
        store(frac.device, sig, best)
    apply(best)
    return best
