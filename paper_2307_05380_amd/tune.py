"""Autotuner for the launch parameters of the graph sweeps.

Tunables (``mg_tuning`` in include/matgraph.h):
- cutoff_wgs_per_cu: persistent workgroups per CU of the cutoff count/fill sweeps;
- cutoff_slots:      destination atoms per lane per image step for structures
                     with more than 64 atoms (1, 2 or 4);
- cutoff_img_group:  image-table entries read per scalar load group by the
                     cutoff sweeps (2, 4 or 8 images per step of the loop);
- knn_wgs_per_cu:    persistent workgroups per CU of the KNN sweep;
- knn_lambda_x4:     4x the expected number of candidates per neighbour that
                     the first KNN search radius is sized for (for cell-list
                     structures it also sets the bin thickness);
- knn_tau_x8:        8x the factor on the uniform-density k-th neighbour
                     distance of the first KNN threshold;
- cutoff_cl_span,
  knn_cl_span:       cell-list stencil half-width in bins (1: 27 bins at least
                     the radius thick; 2: 125 bins at least half of it), tried
                     only when the batch has cell-list structures.

Every candidate is timed with device events over repeated calls and must give
the same graph as the first candidate: the KNN edges bit for bit, the cutoff
edges as a set (the order of a source's edges may depend on the tile shape) with
identical per-source counts and lengths within 2e-5 A (cell-list tiles round
their staged positions relative to the bin, so a length's last bits may depend
on the bin size); the fastest is kept. Results are
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

CUTOFF_SPACE = {"cutoff_wgs_per_cu": [8, 16, 32, 64], "cutoff_slots": [1, 2, 4], "cutoff_img_group": [2, 4, 8]}
KNN_SPACE = {"knn_wgs_per_cu": [2, 4, 8, 16], "knn_lambda_x4": [4, 6, 8, 12], "knn_tau_x8": [9, 10, 12, 16]}
# added when the batch has structures that take cell lists
CL_SPAN_CUTOFF = {"cutoff_cl_span": [1, 2]}
CL_SPAN_KNN = {"knn_cl_span": [1, 2]}


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


def _mix(x: torch.Tensor) -> torch.Tensor:
    """64-bit mixing of int64 values (wrapping arithmetic)."""
    x = x * -7046029254386353131
    x = x ^ (x >> 29)
    return x * -4658895280553007687


def _cutoff_signature(b, count):
    """Per-source edge counts, the edges' identities (src, dst, image) as a sorted
    hash list and their lengths in that order (compared within a tolerance)."""
    E = int(count)
    h = _mix(b.src[:E].long() * 1000003 + b.dst[:E].long())
    for c in range(3):
        h = _mix(h + b.image[:E, c].long() + 7 * (c + 1))
    hs, order = torch.sort(h)
    return [b.row_ptr.clone(), hs, b.length[:E][order].clone()]


def _knn_signature(b):
    return [t.clone() for t in (b.src, b.dst, b.image, b.length)]


def _same(a, b):
    return all(torch.equal(x, y) for x, y in zip(a, b))


def _same_cutoff(a, b, tol: float = 2e-5):
    return (torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
            and (a[2].numel() == 0 or float((a[2] - b[2]).abs().max()) <= tol))


def _clean(rep) -> bool:
    return (rep.flags & ~_lib.MG_FLAG_KNN_EXTENDED) == 0


def tune(lattices, frac, batch_ptr, cutoff: float, k: int, reps: int = 5, space_cutoff=None,
         space_knn=None, verbose: bool = False) -> dict:
    """Time every candidate on this batch; returns {"cutoff": {...}, "knn": {...}, "ms": {...}}."""
    B, N = int(lattices.shape[0]), int(frac.shape[0])
    dev = frac.device
    base = _lib.get_tuning()
    opts = graph.auto_opts(batch_ptr, None)
    big = bool((batch_ptr[1:] - batch_ptr[:-1] >= graph.CL_MIN_ATOMS).any())
    space_cutoff = space_cutoff or dict(CUTOFF_SPACE, **(CL_SPAN_CUTOFF if big else {}))
    space_knn = space_knn or dict(KNN_SPACE, **(CL_SPAN_KNN if big else {}))
    g = graph.cutoff_graph(lattices, frac, batch_ptr, cutoff, opts=opts)
    E, icap = g.num_edges, g.report.images_needed
    del g
    # the first KNN radius (hence the image tables) depends on knn_lambda_x4
    kcap = 1
    for lam in sorted(set(space_knn.get("knn_lambda_x4", [base["knn_lambda_x4"]]))):
        _lib.set_tuning(knn_lambda_x4=lam)
        kcap = max(kcap, graph.knn_graph(lattices, frac, batch_ptr, k, opts=opts).report.images_needed)
    _lib.set_tuning(**base)
    cb = graph.CutoffBuilder(B, N, max(E, 1), max(icap, 1), dev)
    kb = graph.KnnBuilder(B, N, k, max(kcap, 1), dev)
    results = {"cutoff": [], "knn": []}
    ref = None
    for vals in itertools.product(*space_cutoff.values()):
        cfg = dict(zip(space_cutoff.keys(), vals))
        _lib.set_tuning(**cfg)
        ms = _time(lambda: cb.run(lattices, frac, batch_ptr, cutoff, opts), reps)
        snap = _cutoff_signature(cb, E)
        if ref is None:
            ref = snap
        ok = _same_cutoff(ref, snap) and _clean(cb.report())
        results["cutoff"].append((ms, cfg, ok))
        if verbose:
            print("cutoff", cfg, f"{ms:.4f} ms", "ok" if ok else "MISMATCH", flush=True)
    ref = None
    for vals in itertools.product(*space_knn.values()):
        cfg = dict(zip(space_knn.keys(), vals))
        _lib.set_tuning(**cfg)
        ms = _time(lambda: kb.run(lattices, frac, batch_ptr, opts), reps)
        snap = _knn_signature(kb)
        if ref is None:
            ref = snap
        ok = _same(ref, snap) and _clean(kb.report())
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
