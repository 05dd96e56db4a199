"""Torch-facing API over libmatgraph (argument marshalling only).

Every computation runs in the HIP library; torch provides device memory and
the current stream. Tensors must live on a ROCm device:

    lattices  float32 [B, 3, 3]  rows are lattice vectors (Angstrom)
    frac      float32 [N, 3]     fractional coordinates
    batch_ptr int64   [B + 1]    structure b owns atoms batch_ptr[b]:batch_ptr[b+1]

Edges come back as int32 src/dst (global atom indices), int32 image [E, 3]
(the cell of the destination image, Sec. 2.1) and float32 length.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math

import torch

from . import _lib

__all__ = ["Graph", "Report", "cutoff_graph", "knn_graph", "edge_geometry", "EdgeGeometry",
           "CutoffBuilder", "KnnBuilder", "GeometryRunner", "auto_opts", "Triplets", "triplets", "symmetrize",
           "knn_graph_ties", "images_needed", "cutoff_sizes", "CapturedStep"]


@dataclasses.dataclass
class Report:
    num_edges: int
    images_needed: int
    candidates: int
    knn_extended: int
    flags: int

    @staticmethod
    def from_tensor(t: torch.Tensor) -> "Report":
        v = t.cpu().view(torch.int64).tolist()
        return Report(v[0], v[1], v[2], v[3], v[4] & 0xFFFFFFFF)

    def flag_names(self):
        names = {_lib.MG_FLAG_CAPACITY: "capacity", _lib.MG_FLAG_SINGULAR: "singular",
                 _lib.MG_FLAG_NONFINITE: "nonfinite", _lib.MG_FLAG_IMAGES: "images",
                 _lib.MG_FLAG_RANGE: "range", _lib.MG_FLAG_KNN_EXTENDED: "knn_extended",
                 _lib.MG_FLAG_TIES: "ties"}
        return [n for b, n in names.items() if self.flags & b]


@dataclasses.dataclass
class Graph:
    src: torch.Tensor
    dst: torch.Tensor
    image: torch.Tensor
    length: torch.Tensor
    row_ptr: torch.Tensor | None
    report: Report

    @property
    def num_edges(self) -> int:
        return int(self.src.shape[0])


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_inputs(lattices, frac, batch_ptr):
    if not (lattices.is_cuda and frac.is_cuda and batch_ptr.is_cuda):
        raise ValueError("lattices, frac and batch_ptr must be device tensors")
    if lattices.dtype != torch.float32 or frac.dtype != torch.float32:
        raise ValueError("lattices and frac must be float32")
    if batch_ptr.dtype != torch.int64:
        raise ValueError("batch_ptr must be int64")
    if lattices.dim() != 3 or lattices.shape[1:] != (3, 3):
        raise ValueError("lattices must be [B, 3, 3]")
    if frac.dim() != 2 or frac.shape[1] != 3:
        raise ValueError("frac must be [N, 3]")
    B = int(lattices.shape[0])
    if batch_ptr.shape != (B + 1,):
        raise ValueError("batch_ptr must be [B + 1]")
    return lattices.contiguous(), frac.contiguous(), batch_ptr.contiguous(), B, int(frac.shape[0])


CL_MIN_ATOMS = 512   # structures smaller than this never use cell lists (see the C library)


def auto_opts(batch_ptr, opts: int | None = None) -> int:
    """MG_OPT_CELL_LIST_OFF when no structure is large enough for cell lists
    (saves the cell-list launches), else the caller's opts (default 0)."""
    if opts is not None:
        return int(opts)
    counts = batch_ptr[1:] - batch_ptr[:-1]
    nmax = int(counts.max()) if counts.numel() else 0
    return _lib.MG_OPT_CELL_LIST_OFF if nmax < CL_MIN_ATOMS else 0


def _strict_check(rep: Report):
    bad = rep.flags & (_lib.MG_FLAG_SINGULAR | _lib.MG_FLAG_NONFINITE | _lib.MG_FLAG_RANGE)
    if bad:
        raise _lib.MatgraphError(-1, "structures skipped: " + ",".join(rep.flag_names()))


def _radii(r: torch.Tensor, N: int) -> torch.Tensor:
    if not r.is_cuda or r.dtype != torch.float32 or r.shape != (N,):
        raise ValueError(f"per-atom cutoffs must be a float32 device tensor of shape [{N}]")
    return r.contiguous()


class CutoffBuilder:
    """Preallocated cutoff-graph call: fixed batch shape, edge capacity and
    image-table capacity. ``run`` only enqueues kernels (no host sync), so it can
    be replayed or captured into a HIP graph; ``report()`` reads the device
    report (synchronising)."""

    def __init__(self, B: int, N: int, capacity: int, image_capacity: int, device=None,
                 row_ptr: bool = True, vec: bool = False):
        self.lib = _lib.load()
        self.device = torch.device(device or "cuda")
        self.B, self.N = int(B), int(N)
        self.capacity = int(capacity)
        self.image_capacity = int(image_capacity)
        d = self.device
        self.src = torch.empty(self.capacity, dtype=torch.int32, device=d)
        self.dst = torch.empty(self.capacity, dtype=torch.int32, device=d)
        self.image = torch.empty((self.capacity, 3), dtype=torch.int32, device=d)
        self.length = torch.empty(self.capacity, dtype=torch.float32, device=d)
        # edge vectors from the same sweep (mg_cutoff_graph_vec), when asked for
        self.vec = torch.empty((self.capacity, 3), dtype=torch.float32, device=d) if vec else None
        self.row_ptr = torch.empty(self.N + 1, dtype=torch.int64, device=d) if row_ptr else None
        self.rep = torch.zeros(_lib.REPORT_BYTES // 8, dtype=torch.int64, device=d)
        nbytes = self.lib.mg_cutoff_workspace_bytes(self.B, self.N, self.image_capacity)
        self.workspace = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=d)

    def run(self, lattices, frac, batch_ptr, cutoff, opts: int = 0):
        """``cutoff``: one distance (float) or per-atom cutoffs (float32 device tensor [N])."""
        if self.vec is not None:
            radii = _radii(cutoff, self.N) if isinstance(cutoff, torch.Tensor) else None
            _lib.check(self.lib.mg_cutoff_graph_vec(
                _ptr(lattices), _ptr(frac), _ptr(batch_ptr), self.B, self.N,
                1.0 if radii is not None else float(cutoff), _ptr(radii),
                self.capacity, _ptr(self.src), _ptr(self.dst), _ptr(self.image), _ptr(self.length),
                _ptr(self.vec), _ptr(self.row_ptr), _ptr(self.rep), _ptr(self.workspace),
                self.workspace.numel(), int(opts), _stream(self.device)), self.lib)
            return
        if isinstance(cutoff, torch.Tensor):
            radii = _radii(cutoff, self.N)
            _lib.check(self.lib.mg_cutoff_graph_radii(
                _ptr(lattices), _ptr(frac), _ptr(batch_ptr), self.B, self.N, _ptr(radii),
                self.capacity, _ptr(self.src), _ptr(self.dst), _ptr(self.image), _ptr(self.length),
                _ptr(self.row_ptr), _ptr(self.rep), _ptr(self.workspace), self.workspace.numel(),
                int(opts), _stream(self.device)), self.lib)
            return
        _lib.check(self.lib.mg_cutoff_graph(
            _ptr(lattices), _ptr(frac), _ptr(batch_ptr), self.B, self.N, float(cutoff),
            self.capacity, _ptr(self.src), _ptr(self.dst), _ptr(self.image), _ptr(self.length),
            _ptr(self.row_ptr), _ptr(self.rep), _ptr(self.workspace), self.workspace.numel(),
            int(opts), _stream(self.device)), self.lib)

    def report(self) -> Report:
        return Report.from_tensor(self.rep)

    def graph(self, rep: Report | None = None) -> Graph:
        rep = rep or self.report()
        E = min(rep.num_edges, self.capacity)
        return Graph(self.src[:E], self.dst[:E], self.image[:E], self.length[:E], self.row_ptr, rep)

    def overflowed(self, rep: Report | None = None) -> bool:
        """The last run left edges or image slots out (MG_FLAG_CAPACITY / MG_FLAG_IMAGES)."""
        rep = rep or self.report()
        return bool(rep.flags & (_lib.MG_FLAG_CAPACITY | _lib.MG_FLAG_IMAGES))

    def grow(self, rep: Report | None = None, headroom: float = 1.15) -> bool:
        """Reallocate the outputs and the workspace for what the last run
        reported it needs, times ``headroom``. Returns True when anything was
        reallocated (buffers then have new addresses: a captured graph that
        uses them must be captured again)."""
        rep = rep or self.report()
        cap, icap = self.capacity, self.image_capacity
        if rep.flags & _lib.MG_FLAG_CAPACITY:
            cap = max(cap, int(math.ceil(rep.num_edges * headroom)))
        if rep.flags & _lib.MG_FLAG_IMAGES:
            icap = max(icap, int(math.ceil(rep.images_needed * headroom)))
        if cap == self.capacity and icap == self.image_capacity:
            return False
        self.__init__(self.B, self.N, cap, icap, self.device, row_ptr=self.row_ptr is not None,
                      vec=self.vec is not None)
        return True


def cutoff_graph(lattices, frac, batch_ptr, cutoff, capacity: int | None = None,
                 image_capacity: int | None = None, strict: bool = False,
                 opts: int | None = None) -> Graph:
    """Periodic cutoff multigraph (Definition def6, strict <). ``cutoff`` is one
    distance, or a float32 device tensor [N] of per-atom cutoffs c_i (an edge
    uses its source's cutoff).

    Allocates outputs, runs the library and, when the edge or image-table
    capacity was too small, reruns once with the exact sizes the device
    reported (this reads the report, i.e. synchronises)."""
    lattices, frac, batch_ptr, B, N = _check_inputs(lattices, frac, batch_ptr)
    opts = auto_opts(batch_ptr, opts)
    cap = int(capacity) if capacity is not None else max(4096, 96 * N)
    icap = int(image_capacity) if image_capacity is not None else 96 * B + 4096
    for _ in range(3):
        b = CutoffBuilder(B, N, cap, icap, frac.device)
        b.run(lattices, frac, batch_ptr, cutoff, opts)
        rep = b.report()
        retry = False
        if rep.flags & _lib.MG_FLAG_IMAGES:
            icap = int(rep.images_needed)
            retry = True
        if rep.flags & _lib.MG_FLAG_CAPACITY:
            cap = int(rep.num_edges)
            retry = True
        if not retry:
            break
    if strict:
        _strict_check(rep)
    return b.graph(rep)


class KnnBuilder:
    """Preallocated KNN-graph call (output size N*k is fixed)."""

    def __init__(self, B: int, N: int, k: int, image_capacity: int, device=None):
        self.lib = _lib.load()
        self.device = torch.device(device or "cuda")
        self.B, self.N, self.k = int(B), int(N), int(k)
        self.image_capacity = int(image_capacity)
        d = self.device
        M = self.N * self.k
        self.src = torch.empty(M, dtype=torch.int32, device=d)
        self.dst = torch.empty(M, dtype=torch.int32, device=d)
        self.image = torch.empty((M, 3), dtype=torch.int32, device=d)
        self.length = torch.empty(M, dtype=torch.float32, device=d)
        self.rep = torch.zeros(_lib.REPORT_BYTES // 8, dtype=torch.int64, device=d)
        nbytes = self.lib.mg_knn_workspace_bytes(self.B, self.N, self.k, self.image_capacity)
        if nbytes == 0:
            raise ValueError("invalid KNN sizes (k must be in 1..64)")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=d)

    def run(self, lattices, frac, batch_ptr, opts: int = 0):
        _lib.check(self.lib.mg_knn_graph(
            _ptr(lattices), _ptr(frac), _ptr(batch_ptr), self.B, self.N, self.k, _ptr(self.src),
            _ptr(self.dst), _ptr(self.image), _ptr(self.length), _ptr(self.rep),
            _ptr(self.workspace), self.workspace.numel(), int(opts), _stream(self.device)), self.lib)

    def report(self) -> Report:
        return Report.from_tensor(self.rep)

    def graph(self, rep: Report | None = None) -> Graph:
        return Graph(self.src, self.dst, self.image, self.length, None, rep or self.report())

    def overflowed(self, rep: Report | None = None) -> bool:
        """The last run left image slots out (MG_FLAG_IMAGES): some sources are invalid."""
        rep = rep or self.report()
        return bool(rep.flags & _lib.MG_FLAG_IMAGES)

    def grow(self, rep: Report | None = None, headroom: float = 1.15) -> bool:
        """Reallocate the workspace for the image slots the last run needed,
        times ``headroom`` (the output size N*k never changes). Returns True
        when the workspace moved."""
        rep = rep or self.report()
        if not (rep.flags & _lib.MG_FLAG_IMAGES):
            return False
        icap = max(self.image_capacity, int(math.ceil(rep.images_needed * headroom)))
        if icap == self.image_capacity:
            return False
        self.__init__(self.B, self.N, self.k, icap, self.device)
        return True


def knn_graph(lattices, frac, batch_ptr, k: int, image_capacity: int | None = None,
              strict: bool = False, opts: int | None = None) -> Graph:
    """Periodic KNN multigraph: exactly k edges per source in (length, dst, t) order."""
    lattices, frac, batch_ptr, B, N = _check_inputs(lattices, frac, batch_ptr)
    opts = auto_opts(batch_ptr, opts)
    icap = int(image_capacity) if image_capacity is not None else 64 * B + 4096
    for _ in range(3):
        b = KnnBuilder(B, N, k, icap, frac.device)
        b.run(lattices, frac, batch_ptr, opts)
        rep = b.report()
        if rep.flags & _lib.MG_FLAG_IMAGES:
            icap = int(rep.images_needed)
            continue
        break
    if strict:
        _strict_check(rep)
    return b.graph(rep)


def images_needed(lattices, frac, batch_ptr, cutoff=None, k: int = 0, opts: int | None = None) -> Report:
    """Image-table slots a cutoff call (``cutoff``: a distance or per-atom
    float32 device tensor [N]) or a KNN call (``k`` > 0) needs on this batch,
    from the bounds and the batch plan alone (mg_images_needed; synchronises)."""
    lattices, frac, batch_ptr, B, N = _check_inputs(lattices, frac, batch_ptr)
    opts = auto_opts(batch_ptr, opts)
    lib = _lib.load()
    d = frac.device
    radii = None
    if k == 0:
        radii = _radii(cutoff, N) if isinstance(cutoff, torch.Tensor) else None
        nbytes = lib.mg_cutoff_workspace_bytes(B, N, 0)
    else:
        nbytes = lib.mg_knn_workspace_bytes(B, N, int(k), 0)
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=d)
    rep = torch.zeros(_lib.REPORT_BYTES // 8, dtype=torch.int64, device=d)
    _lib.check(lib.mg_images_needed(_ptr(lattices), _ptr(frac), _ptr(batch_ptr), B, N,
                                    1.0 if (radii is not None or k) else float(cutoff), _ptr(radii), int(k),
                                    _ptr(rep), _ptr(ws), ws.numel(), int(opts), _stream(d)), lib)
    return Report.from_tensor(rep)


def cutoff_sizes(lattices, frac, batch_ptr, cutoff, opts: int | None = None) -> tuple[int, int]:
    """(edges, image slots) of the cutoff graph of this batch: the image slots
    from mg_images_needed, then the exact edge count from a cutoff call of
    capacity 0 (count only, no fill). Synchronises; meant for sizing builders
    before a step is captured."""
    lattices, frac, batch_ptr, B, N = _check_inputs(lattices, frac, batch_ptr)
    opts = auto_opts(batch_ptr, opts)
    icap = max(images_needed(lattices, frac, batch_ptr, cutoff, 0, opts).images_needed, 1)
    b = CutoffBuilder(B, N, 0, icap, frac.device)
    b.run(lattices, frac, batch_ptr, cutoff, opts)
    rep = b.report()
    _strict_check(rep)
    return int(rep.num_edges), int(icap)


class CapturedStep:
    """A step of builder calls captured once into a HIP graph and replayed,
    with the overflow protocol a captured call needs: the library never
    allocates, so a replay whose batch needs more edges or image slots than
    the builders hold only sets MG_FLAG_CAPACITY / MG_FLAG_IMAGES (nothing is
    written past a buffer). ``replay(check=True)`` reads the builders' reports
    after the replay (one synchronisation); on an overflow it grows the
    builders that overflowed (``headroom`` times what their report asks for),
    captures the step again and replays it, so the results are complete when
    it returns. ``step`` must enqueue its work on the current stream through
    the builders' ``run`` methods (it is re-run at capture)."""

    def __init__(self, step, builders, headroom: float = 1.15, max_recaptures: int = 4):
        self.step = step
        self.builders = list(builders)
        self.headroom = float(headroom)
        self.max_recaptures = int(max_recaptures)
        self.recaptures = 0
        self.graph = None
        self._capture()

    def _capture(self):
        self.graph = None
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):   # warm-up launch outside the capture
            self.step()
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.step()
        self.graph = g

    def replay(self, check: bool = True) -> bool:
        """Replay the captured step. With ``check``: synchronise, and if a
        builder overflowed, grow it, capture again and replay (up to
        ``max_recaptures`` times). Returns True when the step was captured again."""
        self.graph.replay()
        if not check:
            return False
        again = False
        for _ in range(self.max_recaptures):
            reps = [b.report() for b in self.builders]
            grown = [b.grow(r, self.headroom) for b, r in zip(self.builders, reps) if b.overflowed(r)]
            if not any(grown):
                return again
            self.recaptures += 1
            again = True
            self._capture()
            self.graph.replay()
        raise _lib.MatgraphError(-1, "step still overflows after %d recaptures" % self.max_recaptures)


class GeometryRunner:
    """Preallocated edge-geometry forward / backward for a fixed batch shape.

    The backward pass of a batch with structures of more than 512 atoms runs
    faster with room for its bucket path (16 bytes per edge,
    mg_geometry_backward_workspace_bytes): the runner grows its workspace for
    that on the first backward call with more edges than it has room for
    (``large=None`` reads the batch's largest structure once to decide;
    True / False decide without reading it). Growing reallocates: a captured
    graph that uses the runner must be captured after the first call."""

    def __init__(self, B: int, N: int, device=None, large: bool | None = None):
        self.lib = _lib.load()
        self.device = torch.device(device or "cuda")
        self.B, self.N = int(B), int(N)
        self.large = large
        self.bucket_edges = 0
        nbytes = self.lib.mg_geometry_workspace_bytes(self.B, self.N)
        self.workspace = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)

    def forward(self, lattices, frac, batch_ptr, src, dst, image, vec=None, length=None,
                num_edges=None):
        E = int(src.shape[0])
        _lib.check(self.lib.mg_edge_geometry(
            _ptr(lattices), _ptr(frac), _ptr(batch_ptr), self.B, self.N, _ptr(src), _ptr(dst),
            _ptr(image), E, _ptr(num_edges), _ptr(vec), _ptr(length), _ptr(self.workspace),
            self.workspace.numel(), _stream(self.device)), self.lib)
        return vec, length

    def _room_for_buckets(self, batch_ptr, E: int):
        if self.large is None:
            counts = torch.diff(batch_ptr).max() if self.B > 0 else torch.zeros((), dtype=torch.int64)
            self.large = bool(int(counts) > 512)
        if not self.large or E <= self.bucket_edges:
            return
        nbytes = int(self.lib.mg_geometry_backward_workspace_bytes(self.B, self.N, E))
        if nbytes > self.workspace.numel():
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.bucket_edges = E

    def backward(self, lattices, frac, batch_ptr, src, dst, image, grad_vec=None,
                 grad_length=None, grad_frac=None, grad_lattice=None, num_edges=None):
        E = int(src.shape[0])
        self._room_for_buckets(batch_ptr, E)
        _lib.check(self.lib.mg_edge_geometry_backward(
            _ptr(lattices), _ptr(frac), _ptr(batch_ptr), self.B, self.N, _ptr(src), _ptr(dst),
            _ptr(image), E, _ptr(num_edges), _ptr(grad_vec), _ptr(grad_length), _ptr(grad_frac),
            _ptr(grad_lattice), _ptr(self.workspace), self.workspace.numel(),
            _stream(self.device)), self.lib)
        return grad_frac, grad_lattice


def _edge_inputs(src, dst, image):
    for t, nm in ((src, "src"), (dst, "dst"), (image, "image")):
        if not t.is_cuda or t.dtype != torch.int32:
            raise ValueError(f"{nm} must be an int32 device tensor")
    if image.dim() != 2 or image.shape[1] != 3 or image.shape[0] != src.shape[0] or dst.shape != src.shape:
        raise ValueError("src [E], dst [E], image [E, 3] expected")
    return src.contiguous(), dst.contiguous(), image.contiguous()


class EdgeGeometry(torch.autograd.Function):
    """(vec [E,3], length [E]) of fixed edges, differentiable w.r.t. lattices and frac."""

    @staticmethod
    def forward(ctx, lattices, frac, batch_ptr, src, dst, image):
        lattices, frac, batch_ptr, B, N = _check_inputs(lattices, frac, batch_ptr)
        src, dst, image = _edge_inputs(src, dst, image)
        E = int(src.shape[0])
        run = GeometryRunner(B, N, frac.device)
        vec = torch.empty((E, 3), dtype=torch.float32, device=frac.device)
        length = torch.empty(E, dtype=torch.float32, device=frac.device)
        run.forward(lattices, frac, batch_ptr, src, dst, image, vec, length)
        ctx.save_for_backward(lattices, frac, batch_ptr, src, dst, image)
        ctx.run = run
        return vec, length

    @staticmethod
    def backward(ctx, grad_vec, grad_length):
        lattices, frac, batch_ptr, src, dst, image = ctx.saved_tensors
        need_L, need_x = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gf = torch.empty_like(frac) if need_x else None
        gL = torch.empty_like(lattices) if need_L else None
        if need_x or need_L:
            gv = grad_vec.contiguous().float() if grad_vec is not None else None
            gl = grad_length.contiguous().float() if grad_length is not None else None
            ctx.run.backward(lattices, frac, batch_ptr, src, dst, image, gv, gl, gf, gL)
        return gL, gf, None, None, None, None


def edge_geometry(lattices, frac, batch_ptr, src, dst, image):
    """Differentiable (vec, length) of the given edges (see ``EdgeGeometry``)."""
    return EdgeGeometry.apply(lattices, frac, batch_ptr, src, dst, image)


@dataclasses.dataclass
class Triplets:
    e1: torch.Tensor           # int32 [T] first edge of each pair
    e2: torch.Tensor           # int32 [T] second edge (same source, e2 != e1)
    cos_theta: torch.Tensor | None
    trip_ptr: torch.Tensor     # int64 [N+1]
    report: Report


def triplets(row_ptr: torch.Tensor, num_edges: int, vec: torch.Tensor | None = None,
             capacity: int | None = None) -> Triplets:
    """Ordered pairs of different edges sharing a source (Definition def6,
    Gamma_2) for a graph grouped by source (``row_ptr`` int64 [N+1] on the
    device), with the angle between the edge vectors when ``vec`` [E,3] is
    given. Reruns once with the exact size when ``capacity`` was too small."""
    if not row_ptr.is_cuda or row_ptr.dtype != torch.int64 or row_ptr.dim() != 1:
        raise ValueError("row_ptr must be an int64 device tensor [N+1]")
    lib = _lib.load()
    d = row_ptr.device
    N = int(row_ptr.shape[0]) - 1
    E = int(num_edges)
    if vec is not None:
        if vec.dtype != torch.float32 or vec.shape != (E, 3) or not vec.is_cuda:
            raise ValueError(f"vec must be a float32 device tensor [{E}, 3]")
        vec = vec.contiguous()
    row_ptr = row_ptr.contiguous()
    cap = int(capacity) if capacity is not None else max(1024, 16 * E)
    ws = torch.empty(max(int(lib.mg_triplets_workspace_bytes(N)), 256), dtype=torch.uint8, device=d)
    rep_t = torch.zeros(_lib.REPORT_BYTES // 8, dtype=torch.int64, device=d)
    trip_ptr = torch.empty(N + 1, dtype=torch.int64, device=d)
    for _ in range(2):
        e1 = torch.empty(cap, dtype=torch.int32, device=d)
        e2 = torch.empty(cap, dtype=torch.int32, device=d)
        cs = torch.empty(cap, dtype=torch.float32, device=d) if vec is not None else None
        _lib.check(lib.mg_triplets(_ptr(row_ptr), N, E, _ptr(vec), cap, _ptr(e1), _ptr(e2), _ptr(cs),
                                   _ptr(trip_ptr), _ptr(rep_t), _ptr(ws), ws.numel(), _stream(d)), lib)
        rep = Report.from_tensor(rep_t)
        if rep.flags & _lib.MG_FLAG_CAPACITY:
            cap = int(rep.num_edges)
            continue
        break
    T = min(rep.num_edges, cap)
    return Triplets(e1[:T], e2[:T], cs[:T] if cs is not None else None, trip_ptr, rep)


def symmetrize(row_ptr: torch.Tensor, dst: torch.Tensor, image: torch.Tensor,
               length: torch.Tensor | None = None, capacity: int | None = None) -> Graph:
    """Symmetric closure of a graph grouped by source (``row_ptr`` int64 [N+1],
    ``dst`` int32 [E], ``image`` int32 [E,3], optional ``length`` [E]): adds
    every missing reverse edge (j, i, -t) once, with the same length. For a
    KNN graph pass ``row_ptr = arange(0, N*k + 1, k)``."""
    if not row_ptr.is_cuda or row_ptr.dtype != torch.int64 or row_ptr.dim() != 1:
        raise ValueError("row_ptr must be an int64 device tensor [N+1]")
    E = int(dst.shape[0])
    for t, nm in ((dst, "dst"), (image, "image")):
        if not t.is_cuda or t.dtype != torch.int32:
            raise ValueError(f"{nm} must be an int32 device tensor")
    if image.shape != (E, 3):
        raise ValueError("image must be [E, 3]")
    if length is not None and (length.dtype != torch.float32 or length.shape != (E,)):
        raise ValueError("length must be float32 [E]")
    lib = _lib.load()
    d = row_ptr.device
    N = int(row_ptr.shape[0]) - 1
    row_ptr, dst, image = row_ptr.contiguous(), dst.contiguous(), image.contiguous()
    length = length.contiguous() if length is not None else None
    cap = int(capacity) if capacity is not None else 2 * E
    ws = torch.empty(max(int(lib.mg_symmetrize_workspace_bytes(N, E)), 256), dtype=torch.uint8, device=d)
    rep_t = torch.zeros(_lib.REPORT_BYTES // 8, dtype=torch.int64, device=d)
    out_ptr = torch.empty(N + 1, dtype=torch.int64, device=d)
    for _ in range(2):
        s_ = torch.empty(cap, dtype=torch.int32, device=d)
        d_ = torch.empty(cap, dtype=torch.int32, device=d)
        i_ = torch.empty((cap, 3), dtype=torch.int32, device=d)
        l_ = torch.empty(cap, dtype=torch.float32, device=d) if length is not None else None
        _lib.check(lib.mg_symmetrize(_ptr(row_ptr), N, _ptr(dst), _ptr(image), _ptr(length), E, cap, _ptr(s_),
                                     _ptr(d_), _ptr(i_), _ptr(l_), _ptr(out_ptr), _ptr(rep_t), _ptr(ws),
                                     ws.numel(), _stream(d)), lib)
        rep = Report.from_tensor(rep_t)
        if rep.flags & _lib.MG_FLAG_CAPACITY:
            cap = int(rep.num_edges)
            continue
        break
    S = min(rep.num_edges, cap)
    return Graph(s_[:S], d_[:S], i_[:S], l_[:S] if l_ is not None else None, out_ptr, rep)


def knn_graph_ties(lattices, frac, batch_ptr, k: int, capacity: int | None = None,
                   image_capacity: int | None = None, opts: int | None = None) -> Graph:
    """KNN multigraph with ties at the k-th distance kept (Algorithm 2's d <= d_k):
    variable edges per source, grouped by source (row_ptr), in (length, dst, t)
    order. Reruns with the exact sizes when a capacity was too small."""
    lattices, frac, batch_ptr, B, N = _check_inputs(lattices, frac, batch_ptr)
    opts = auto_opts(batch_ptr, opts)
    lib = _lib.load()
    d = frac.device
    cap = int(capacity) if capacity is not None else max(1024, N * (int(k) + 8))
    icap = int(image_capacity) if image_capacity is not None else 64 * B + 4096
    rep_t = torch.zeros(_lib.REPORT_BYTES // 8, dtype=torch.int64, device=d)
    row_ptr = torch.empty(N + 1, dtype=torch.int64, device=d)
    for _ in range(3):
        nbytes = lib.mg_knn_ties_workspace_bytes(B, N, int(k), icap)
        if nbytes == 0:
            raise ValueError("invalid sizes (k must be in 1..63)")
        ws = torch.empty(int(nbytes), dtype=torch.uint8, device=d)
        s_ = torch.empty(cap, dtype=torch.int32, device=d)
        d_ = torch.empty(cap, dtype=torch.int32, device=d)
        i_ = torch.empty((cap, 3), dtype=torch.int32, device=d)
        l_ = torch.empty(cap, dtype=torch.float32, device=d)
        _lib.check(lib.mg_knn_graph_ties(_ptr(lattices), _ptr(frac), _ptr(batch_ptr), B, N, int(k), cap, _ptr(s_),
                                         _ptr(d_), _ptr(i_), _ptr(l_), _ptr(row_ptr), _ptr(rep_t), _ptr(ws),
                                         ws.numel(), int(opts), _stream(d)), lib)
        rep = Report.from_tensor(rep_t)
        retry = False
        if rep.flags & _lib.MG_FLAG_IMAGES:
            icap = int(rep.images_needed)
            retry = True
        if rep.flags & _lib.MG_FLAG_CAPACITY:
            cap = int(rep.num_edges)
            retry = True
        if not retry:
            break
    E = min(rep.num_edges, cap)
    return Graph(s_[:E], d_[:E], i_[:E], l_[:E], row_ptr, rep)
