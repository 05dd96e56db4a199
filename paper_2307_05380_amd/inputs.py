"""Seeded synthetic crystal batches.

This module only draws inputs: lattices, fractional coordinates, batch
pointers and the random weights of the differentiation workload. It contains
none of the graph method's arithmetic, so both the HIP path and the FP64
oracle can consume its output without sharing any code.

Materials are triples (rho, x, z) of a lattice, fractional coordinates in
[0, 1)^{n x 3} and features (Sec. 2.1, Definition "featured materials"). The
feature sequence z is never read by graph construction and is not generated.
Lattices are returned with the lattice vectors as ROWS: ``L[b, k]`` is the
k-th lattice vector in Angstrom, so a Cartesian position is ``frac @ L``.

Five workloads are provided. The paper's dataset (Materials Project filtered
to at most 64 atoms per structure, Sec. 3) is not available; these seeded
batches stand in for it with the sizes, skew and atom-count mixes listed in
each ``make_config*`` docstring.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 230705380

__all__ = [
    "Batch",
    "SEED_BASE",
    "cell_from_parameters",
    "volume_factor",
    "make_config",
    "make_config1",
    "make_config2",
    "make_config3",
    "make_config4",
    "make_config5",
    "config5_step_delta",
    "loss_weights",
    "random_batch",
]


@dataclasses.dataclass
class Batch:
    """A batch of structures in the layout the library consumes.

    lattices:  float32 [B, 3, 3], rows are lattice vectors (Angstrom)
    frac:      float32 [N, 3] fractional coordinates
    batch_ptr: int64 [B + 1], structure b owns atoms batch_ptr[b]:batch_ptr[b+1]
    cutoff:    cutoff radius in Angstrom used by the workload
    k:         number of neighbours used by the workload's KNN graph
    """

    lattices: np.ndarray
    frac: np.ndarray
    batch_ptr: np.ndarray
    cutoff: float
    k: int
    name: str = ""

    @property
    def B(self) -> int:
        return int(self.lattices.shape[0])

    @property
    def N(self) -> int:
        return int(self.frac.shape[0])

    def counts(self) -> np.ndarray:
        return np.diff(self.batch_ptr)

    def structure(self, b: int):
        """(lattice [3,3] f32, frac [n,3] f32) of structure b."""
        a, e = int(self.batch_ptr[b]), int(self.batch_ptr[b + 1])
        return self.lattices[b], self.frac[a:e]

    def subset(self, idx) -> "Batch":
        """A new batch holding the structures listed in ``idx`` (in order)."""
        idx = [int(i) for i in idx]
        lat = self.lattices[idx].copy()
        parts = [self.frac[self.batch_ptr[i]:self.batch_ptr[i + 1]] for i in idx]
        frac = np.concatenate(parts, 0) if parts else np.zeros((0, 3), np.float32)
        ptr = np.zeros(len(idx) + 1, np.int64)
        ptr[1:] = np.cumsum([len(p) for p in parts])
        return Batch(lat, np.ascontiguousarray(frac, np.float32), ptr, self.cutoff, self.k,
                     self.name + "[subset]")


def volume_factor(alpha: float, beta: float, gamma: float) -> float:
    """sqrt(1 - cos^2 a - cos^2 b - cos^2 g + 2 cos a cos b cos g); NaN if not realisable.

    The volume of a cell with unit edge lengths and these angles (radians).
    Used to reject nearly degenerate angle draws.
    """
    ca, cb, cg = math.cos(alpha), math.cos(beta), math.cos(gamma)
    q = 1.0 - ca * ca - cb * cb - cg * cg + 2.0 * ca * cb * cg
    return math.sqrt(q) if q > 0.0 else float("nan")


def cell_from_parameters(a: float, b: float, c: float, alpha: float, beta: float,
                         gamma: float) -> np.ndarray:
    """Lower-triangular row-vector lattice from lengths and angles (radians), FP64.

    a1 = (a, 0, 0); a2 = (b cos g, b sin g, 0);
    a3 = (c cos b, c (cos a - cos b cos g) / sin g, c * sqrt(rest)).
    """
    ca, cb, cg, sg = math.cos(alpha), math.cos(beta), math.cos(gamma), math.sin(gamma)
    c2 = (ca - cb * cg) / sg
    c3 = math.sqrt(max(1.0 - cb * cb - c2 * c2, 0.0))
    return np.array([[a, 0.0, 0.0],
                     [b * cg, b * sg, 0.0],
                     [c * cb, c * c2, c * c3]], dtype=np.float64)


def _draw_cell(rng, len_lo, len_hi, ang_lo_deg, ang_hi_deg, min_vf=0.05):
    lengths = rng.uniform(len_lo, len_hi, size=3)
    while True:
        ang = np.deg2rad(rng.uniform(ang_lo_deg, ang_hi_deg, size=3))
        vf = volume_factor(*ang)
        if vf == vf and vf >= min_vf:
            break
    return cell_from_parameters(*lengths, *ang)


def _pack(lats, fracs, cutoff, k, name) -> Batch:
    ptr = np.zeros(len(fracs) + 1, np.int64)
    ptr[1:] = np.cumsum([f.shape[0] for f in fracs])
    frac = np.concatenate(fracs, 0).astype(np.float32) if fracs else np.zeros((0, 3), np.float32)
    lat = np.stack(lats, 0).astype(np.float32)
    return Batch(np.ascontiguousarray(lat), np.ascontiguousarray(frac), ptr, float(cutoff), int(k), name)


def make_config1(seed: int | None = None) -> Batch:
    """Single structure: 16 atoms, L = 5 (I + U(-0.1, 0.1)^{3x3}), cutoff 6 A, k = 12."""
    rng = np.random.default_rng(SEED_BASE + 1 if seed is None else seed)
    L = 5.0 * (np.eye(3) + rng.uniform(-0.1, 0.1, size=(3, 3)))
    x = rng.random((16, 3), dtype=np.float32)
    return _pack([L], [x], 6.0, 12, "config1")


def _uniform_batch(rng, B, n_lo, n_hi, len_lo, len_hi, ang_lo, ang_hi):
    lats, fracs = [], []
    for _ in range(B):
        n = int(rng.integers(n_lo, n_hi + 1))
        L = _draw_cell(rng, len_lo, len_hi, ang_lo, ang_hi)
        lats.append(L)
        fracs.append(rng.random((n, 3), dtype=np.float32))
    return lats, fracs


def make_config2(seed: int | None = None, B: int = 256) -> Batch:
    """256 structures: n ~ U{4..64}, lengths U(3, 15) A, angles U(60, 120) deg; cutoff 6, k = 16."""
    rng = np.random.default_rng(SEED_BASE + 2 if seed is None else seed)
    lats, fracs = _uniform_batch(rng, B, 4, 64, 3.0, 15.0, 60.0, 120.0)
    return _pack(lats, fracs, 6.0, 16, "config2")


def make_config3(seed: int | None = None, B: int = 4096) -> Batch:
    """4096 structures, n = floor(exp(U(0, ln 129))) in 1..128 (log-uniform), lengths
    U(2.5, 20) A, angles U(30, 150) deg with volume factor >= 0.05; cutoff 8 A, k = 16."""
    rng = np.random.default_rng(SEED_BASE + 3 if seed is None else seed)
    lats, fracs = [], []
    for _ in range(B):
        n = int(math.floor(math.exp(rng.uniform(0.0, math.log(129.0)))))
        n = min(max(n, 1), 128)
        L = _draw_cell(rng, 2.5, 20.0, 30.0, 150.0)
        lats.append(L)
        fracs.append(rng.random((n, 3), dtype=np.float32))
    return _pack(lats, fracs, 8.0, 16, "config3")


def make_config4(seed: int | None = None, B: int = 1024) -> Batch:
    """1024 structures drawn as in the 256-structure batch; cutoff 6 A (differentiation)."""
    rng = np.random.default_rng(SEED_BASE + 4 if seed is None else seed)
    lats, fracs = _uniform_batch(rng, B, 4, 64, 3.0, 15.0, 60.0, 120.0)
    return _pack(lats, fracs, 6.0, 16, "config4")


def make_config5(seed: int | None = None, B: int = 64, m_lo: int = 8, m_hi: int = 16) -> Batch:
    """64 supercells: an 8-atom base cell (lengths U(3, 5) A, angles U(80, 100) deg,
    frac U[0,1)) tiled m x m x m with m ~ U{8..16}, then every atom displaced by a
    Cartesian N(0, 0.05 A) draw mapped to fractional coordinates with the FP64
    inverse of the supercell. Cutoff 5 A, k = 32. Coordinates are not wrapped."""
    rng = np.random.default_rng(SEED_BASE + 5 if seed is None else seed)
    lats, fracs = [], []
    for _ in range(B):
        base = _draw_cell(rng, 3.0, 5.0, 80.0, 100.0)
        xb = rng.random((8, 3), dtype=np.float32).astype(np.float64)
        m = int(rng.integers(m_lo, m_hi + 1))
        g = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1)
        g = g.reshape(-1, 3).astype(np.float64)
        x = ((g[:, None, :] + xb[None, :, :]) / m).reshape(-1, 3)
        L = base * m
        disp = rng.normal(0.0, 0.05, size=x.shape) @ np.linalg.inv(L)
        lats.append(L)
        fracs.append((x + disp).astype(np.float32))
    return _pack(lats, fracs, 5.0, 32, "config5")


def config5_step_delta(batch: Batch, step: int, sigma: float = 0.02, seed: int | None = None) -> np.ndarray:
    """Fractional-coordinate increment [N, 3] f32 for update step ``step``: a Cartesian
    N(0, sigma) draw per atom mapped through the FP64 inverse of its lattice."""
    rng = np.random.default_rng((SEED_BASE + 50 if seed is None else seed) * 1000 + step)
    out = np.empty((batch.N, 3), np.float64)
    for b in range(batch.B):
        a, e = int(batch.batch_ptr[b]), int(batch.batch_ptr[b + 1])
        Linv = np.linalg.inv(batch.lattices[b].astype(np.float64))
        out[a:e] = rng.normal(0.0, sigma, size=(e - a, 3)) @ Linv
    return out.astype(np.float32)


def make_config(i: int, seed: int | None = None, **kw) -> Batch:
    return {1: make_config1, 2: make_config2, 3: make_config3, 4: make_config4,
            5: make_config5}[int(i)](seed, **kw)


def loss_weights(num_edges: int, seed: int = SEED_BASE + 40) -> np.ndarray:
    """w_e ~ N(0, 1) float32 for the differentiation loss, one per edge in
    canonical (src, dst, t) order."""
    return np.random.default_rng(seed).standard_normal(num_edges).astype(np.float32)


def random_batch(rng, B, n_lo, n_hi, len_lo=2.5, len_hi=12.0, ang_lo=40.0, ang_hi=140.0,
                 cutoff=5.0, k=8, min_vf=0.05, name="random") -> Batch:
    """Small random batch for tests: uniform atom counts and cell parameters."""
    lats, fracs = [], []
    for _ in range(B):
        n = int(rng.integers(n_lo, n_hi + 1))
        lats.append(_draw_cell(rng, len_lo, len_hi, ang_lo, ang_hi, min_vf))
        fracs.append(rng.random((n, 3), dtype=np.float32))
    return _pack(lats, fracs, cutoff, k, name)
