"""FP64 brute-force cutoff and KNN multigraphs (oracle; test infrastructure only).

What is computed (paper Sec. 2.1, Definition def6):

    Gamma_1 = {(i, j, t) in Gamma_0 x Gamma_0 x Z^3 : || (x_j - x_i + t) L || < c_i}

with c_i the cutoff of the source atom (one constant c for every atom in the
common case), minus the self-image (i, i, 0). Because a periodic crystal is a multigraph
(Sec. 1), a pair (i, j) may carry several edges, and an atom has edges to its
own images (i, i, t != 0).

The KNN graph is the same definition with c_i set per source so that exactly
the k nearest (j, t) are kept (Sec. 1 and the remark after Definition def6).
Ties are ordered by the key (length, dst, t0, t1, t2), all ascending.

Bounded enumeration. With f = x_j - x_i + t and v = f L, one has f = v L^{-1},
so |f_k| = |v . (L^{-1})[:, k]| <= ||v|| * r_k where r_k is the norm of
column k of L^{-1} (Cauchy-Schwarz). Every candidate with ||v|| <= R
therefore has t_k in [ceil(-R r_k - d_k), floor(R r_k - d_k)], d = x_j - x_i.
This plays the role of the paper's test that the region of cells evaluated
covers the search sphere (Sec. 2.2, Fig. 2). The oracle enumerates the union of those ranges over
all destinations of one source and tests every candidate; the KNN search
grows R (doubling) until the k-th distance is covered, which is Algorithm 1's
expanding search used only as a bound.

Nothing is wrapped or reordered: coordinates are used as given (values
outside [0, 1) are allowed; t is relative to the given x).

Parity status: pinned. Closed-form coordination numbers (sc/bcc/fcc),
sums of three squares for the simple cubic lattice, the row-vector convention
pin, edge symmetry, supercell and unimodular-basis invariance, translation
invariance, KNN-vs-cutoff consistency and an enormous-image-range brute force
on tiny cells are checked by the CPU tests.
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

# Slack on the integer image bounds. The bound itself is exact; FP64 rounding
# of R * r_k - d_k is ~1e-15, far below this.
_BOX_SLACK = 1e-9


@dataclasses.dataclass
class Graph64:
    """Edges with global atom indices: int64 src/dst, int64 image [E, 3], float64 length."""

    src: np.ndarray
    dst: np.ndarray
    image: np.ndarray
    length: np.ndarray

    @property
    def num_edges(self) -> int:
        return int(self.src.shape[0])


@dataclasses.dataclass
class KnnResult64:
    """KNN oracle result.

    graph:  the k selected edges of every source, source-major, each source's
            k edges in key order (length, dst, t0, t1, t2).
    dk:     float64 [N] k-th distance of every source.
    near:   dict source -> list of (dst, t0, t1, t2, length) candidates with
            |length - dk| <= band (only filled when band > 0).
    inside: int64 [N] number of selected edges with length < dk - band.
    """

    graph: Graph64
    dk: np.ndarray
    near: dict
    inside: np.ndarray


def inverse_column_norms64(L: np.ndarray) -> np.ndarray:
    """r_k = || column k of L^{-1} || with L^{-1} from numpy.linalg.inv (FP64)."""
    Li = np.linalg.inv(np.asarray(L, np.float64))
    return np.sqrt((Li * Li).sum(axis=0))


def image_ranges64(L: np.ndarray, d: np.ndarray, R: float):
    """Integer ranges [lo, hi] (per row of d) holding every t with ||(d + t) L|| <= R."""
    r = inverse_column_norms64(L)
    d = np.asarray(d, np.float64)
    lo = np.ceil(-R * r - d - _BOX_SLACK).astype(np.int64)
    hi = np.floor(R * r - d + _BOX_SLACK).astype(np.int64)
    return lo, hi


def _grid(lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    axes = [np.arange(int(lo[k]), int(hi[k]) + 1, dtype=np.int64) for k in range(3)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)
    return g.reshape(-1, 3)


def _candidates_within(L: np.ndarray, x: np.ndarray, i: int, R: float):
    """All (j, t, length) from source i with length <= R, self-image excluded.

    Returns (j [M], t [M,3], length [M]) in no particular order.
    """
    d = x - x[i]                                   # x_j - x_i, [n, 3]
    lo, hi = image_ranges64(L, d, R)
    T = _grid(lo.min(axis=0), hi.max(axis=0))      # union of the per-pair ranges
    f = d[:, None, :] + T[None, :, :].astype(np.float64)   # [n, T, 3]
    v = f @ L
    length = np.sqrt((v * v).sum(axis=-1))
    keep = length <= R
    self_t = np.nonzero((T == 0).all(axis=1))[0]
    if self_t.size:
        keep[i, self_t[0]] = False
    jj, tt = np.nonzero(keep)
    return jj.astype(np.int64), T[tt], length[jj, tt]


def cutoff_structure64(L, x, cutoff, band: float = 0.0):
    """Edges of one structure with length < c_src + band, sorted by (src, dst, t).

    ``cutoff`` is one distance for every atom, or an array of per-atom cutoffs
    c_i (the cutoff of an edge is its source's, Definition def6). Returns local
    (src, dst, image [E,3], length) arrays; with band = 0 this is exactly
    Definition def6.
    """
    return cutoff_sources64(L, x, cutoff, range(np.asarray(x).shape[0]), band)


def cutoff_sources64(L, x, cutoff, sources, band: float = 0.0):
    """Edges of the listed sources of one structure with length < c_src + band
    (same definition as ``cutoff_structure64``, restricted to some sources, for
    structures too large to enumerate whole). Sorted by (src, dst, t)."""
    L = np.asarray(L, np.float64)
    x = np.asarray(x, np.float64)
    radii = np.broadcast_to(np.asarray(cutoff, np.float64), (x.shape[0],))
    out = [[], [], [], []]
    for i in sources:
        R = float(radii[int(i)]) + float(band)
        j, t, length = _candidates_within(L, x, int(i), R)
        m = length < R
        out[0].append(np.full(int(m.sum()), int(i), np.int64))
        out[1].append(j[m])
        out[2].append(t[m])
        out[3].append(length[m])
    if not out[0]:
        return (np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 3), np.int64), np.zeros(0))
    src, dst = np.concatenate(out[0]), np.concatenate(out[1])
    img, length = np.concatenate(out[2]).reshape(-1, 3), np.concatenate(out[3])
    order = np.lexsort((img[:, 2], img[:, 1], img[:, 0], dst, src))
    return src[order], dst[order], img[order], length[order]


def knn_structure64(L, x, k: int, band: float = 0.0, sources=None):
    """k nearest (j, t) of every source of one structure (Sec. 1, Definition def6 remark).

    Returns (src, dst, image, length, dk, near, inside) with local indices;
    each source's k edges are in key order (length, dst, t0, t1, t2).
    ``sources`` restricts the computation to some sources (rows in that order).
    """
    L = np.asarray(L, np.float64)
    x = np.asarray(x, np.float64)
    n = x.shape[0]
    vol = abs(float(np.linalg.det(L)))
    R0 = (3.0 * (k + 1) * vol / (4.0 * math.pi * max(n, 1))) ** (1.0 / 3.0)
    srcs = list(range(n)) if sources is None else [int(i) for i in sources]
    ns = len(srcs)
    src = np.zeros(ns * k, np.int64)
    dst = np.zeros(ns * k, np.int64)
    img = np.zeros((ns * k, 3), np.int64)
    length = np.zeros(ns * k, np.float64)
    dk = np.zeros(ns, np.float64)
    inside = np.zeros(ns, np.int64)
    near = {}
    for r, i in enumerate(srcs):
        R = R0
        while True:
            j, t, ln = _candidates_within(L, x, i, R)
            if ln.shape[0] >= k:
                order = np.lexsort((t[:, 2], t[:, 1], t[:, 0], j, ln))
                d = ln[order[k - 1]]
                if d + band <= R:
                    break
                R = d + band          # every candidate up to d + band is then enumerated
            else:
                R = 2.0 * R           # extend the search area (Algorithm 1)
        sel = order[:k]
        src[r * k:(r + 1) * k] = i
        dst[r * k:(r + 1) * k] = j[sel]
        img[r * k:(r + 1) * k] = t[sel]
        length[r * k:(r + 1) * k] = ln[sel]
        dk[r] = d
        inside[r] = int((ln[sel] < d - band).sum())
        if band > 0.0:
            m = np.abs(ln - d) <= band
            near[i] = [(int(a), int(b[0]), int(b[1]), int(b[2]), float(c))
                       for a, b, c in zip(j[m], t[m], ln[m])]
    return src, dst, img, length, dk, near, inside


def knn_ties_structure64(L, x, k: int, sources=None):
    """Algorithm 2's selection with ties kept: every (j, t) of a source whose
    length is <= the source's k-th distance d_k (Sec. 2.2), so a source can get
    more than k edges when several candidates share the k-th distance.

    Returns (src, dst, image, length, row_ptr) with local indices, each source's
    edges in key order (length, dst, t0, t1, t2).
    """
    L = np.asarray(L, np.float64)
    x = np.asarray(x, np.float64)
    srcs = list(range(x.shape[0])) if sources is None else [int(i) for i in sources]
    _, _, _, _, dk, _, _ = knn_structure64(L, x, k, sources=srcs)
    out = [[], [], [], []]
    ptr = [0]
    for r, i in enumerate(srcs):
        j, t, ln = _candidates_within(L, x, i, float(dk[r]))
        keep = ln <= dk[r]
        j, t, ln = j[keep], t[keep], ln[keep]
        by_key = np.lexsort((t[:, 2], t[:, 1], t[:, 0], j, ln))      # (length, dst, t0, t1, t2)
        out[0].append(np.full(by_key.shape[0], i, np.int64))
        out[1].append(j[by_key])
        out[2].append(t[by_key])
        out[3].append(ln[by_key])
        ptr.append(ptr[-1] + by_key.shape[0])
    if not srcs:
        z = np.zeros(0, np.int64)
        return z, z, np.zeros((0, 3), np.int64), np.zeros(0), np.zeros(1, np.int64)
    return (np.concatenate(out[0]), np.concatenate(out[1]), np.concatenate(out[2]).reshape(-1, 3),
            np.concatenate(out[3]), np.asarray(ptr, np.int64))


def _structure_slices(batch_ptr, structures):
    ptr = np.asarray(batch_ptr, np.int64)
    if structures is None:
        structures = range(ptr.shape[0] - 1)
    return [(int(s), int(ptr[s]), int(ptr[s + 1])) for s in structures]


def _cutoff_task(args):
    L, x, cutoff, band, base = args
    s, d, t, ln = cutoff_structure64(L, x, cutoff, band)
    return s + base, d + base, t, ln


def _knn_task(args):
    L, x, k, band, base = args
    s, d, t, ln, dk, near, inside = knn_structure64(L, x, k, band)
    near = {i + base: [(a + base,) + tuple(rest) for (a, *rest) in v] for i, v in near.items()}
    return s + base, d + base, t, ln, dk, near, inside


def _run(task, jobs, processes):
    if processes is None:
        processes = 1
    if processes <= 1 or len(jobs) <= 1:
        return [task(j) for j in jobs]
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(processes, initializer=_single_thread_blas) as pool:
        return pool.map(task, jobs, chunksize=max(1, len(jobs) // (8 * processes)))


def _single_thread_blas():
    for var in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var] = "1"


def cutoff_graph64(lattices, frac, batch_ptr, cutoff, band: float = 0.0,
                   structures=None, processes: int | None = None) -> Graph64:
    """Cutoff multigraph of a batch (global atom indices), structure-major, each
    structure's edges sorted by (src, dst, t). ``cutoff`` is a scalar or an
    array [N] of per-atom cutoffs. ``structures`` restricts the computation to a
    subset of structure indices (in the given order)."""
    lattices = np.asarray(lattices, np.float64)
    frac = np.asarray(frac, np.float64)
    radii = np.broadcast_to(np.asarray(cutoff, np.float64), (frac.shape[0],))
    jobs = [(lattices[s], frac[a:e], radii[a:e], band, a)
            for s, a, e in _structure_slices(batch_ptr, structures)]
    parts = _run(_cutoff_task, jobs, processes)
    if not parts:
        return Graph64(np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros((0, 3), np.int64),
                       np.zeros(0))
    return Graph64(np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]),
                   np.concatenate([p[2] for p in parts]).reshape(-1, 3),
                   np.concatenate([p[3] for p in parts]))


def knn_graph64(lattices, frac, batch_ptr, k: int, band: float = 0.0, structures=None,
                processes: int | None = None) -> KnnResult64:
    """KNN multigraph of a batch: k edges per source in key order (global indices)."""
    lattices = np.asarray(lattices, np.float64)
    frac = np.asarray(frac, np.float64)
    jobs = [(lattices[s], frac[a:e], k, band, a)
            for s, a, e in _structure_slices(batch_ptr, structures)]
    parts = _run(_knn_task, jobs, processes)
    near = {}
    for p in parts:
        near.update(p[5])
    if not parts:
        z = np.zeros(0, np.int64)
        return KnnResult64(Graph64(z, z, np.zeros((0, 3), np.int64), np.zeros(0)), np.zeros(0), {}, z)
    g = Graph64(np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts]),
                np.concatenate([p[2] for p in parts]).reshape(-1, 3),
                np.concatenate([p[3] for p in parts]))
    return KnnResult64(g, np.concatenate([p[4] for p in parts]), near,
                       np.concatenate([p[6] for p in parts]))
