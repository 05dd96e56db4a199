"""FP64 edge geometry, its vector-Jacobian product and finite differences
(oracle; test infrastructure only).

Edge vector and length follow the norm inside Definition def6 (Sec. 2.1):
v_e = (x_dst - x_src + t_e) L_s and l_e = ||v_e||, with L_s the lattice of the
structure that owns the source atom (rows are lattice vectors).

The backward pass is what lets a generative model move the geometry and
rebuild the graph inside its forward pass (abstract; Sec. 4): with the edge
set held fixed and upstream gradients (g_v, g_l),

    g_e            = g_v,e + g_l,e * v_e / l_e        (0 * v / l := 0 when l_e = 0)
    grad_x[dst_e] += g_e L_s^T
    grad_x[src_e] -= g_e L_s^T
    grad_L[s]     += f_e^T g_e,   f_e = x_dst - x_src + t_e

Parity status: pinned. ``fd_vjp64`` (central differences of the scalar
J = sum_e g_v,e . v_e + g_l,e l_e, which uses only the forward) checks the
analytic product; the CPU tests also check sum_i grad_x[i] = 0 per structure,
the symmetry of L^T G_L for length-only losses and tr(L^T G_L) = sum_e l_e g_l,e.
"""
from __future__ import annotations

import numpy as np


def _structure_of(batch_ptr, atoms):
    return np.searchsorted(np.asarray(batch_ptr, np.int64), np.asarray(atoms, np.int64),
                           side="right") - 1


def _frac_displacement(frac, src, dst, image):
    frac = np.asarray(frac, np.float64)
    return frac[np.asarray(dst)] - frac[np.asarray(src)] + np.asarray(image, np.float64)


def edge_geometry64(lattices, frac, batch_ptr, src, dst, image):
    """(vec [E,3], length [E]) in FP64."""
    lattices = np.asarray(lattices, np.float64)
    s = _structure_of(batch_ptr, src)
    f = _frac_displacement(frac, src, dst, image)
    v = np.einsum("ek,ekm->em", f, lattices[s]) if f.shape[0] else np.zeros((0, 3))
    return v, np.sqrt((v * v).sum(axis=1))


def edge_geometry_vjp64(lattices, frac, batch_ptr, src, dst, image, grad_vec=None,
                        grad_len=None):
    """(grad_frac [N,3], grad_lattice [B,3,3]) of the edge geometry for the given
    upstream gradients (either may be None)."""
    lattices = np.asarray(lattices, np.float64)
    frac = np.asarray(frac, np.float64)
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    v, length = edge_geometry64(lattices, frac, batch_ptr, src, dst, image)
    g = np.zeros_like(v)
    if grad_vec is not None:
        g += np.asarray(grad_vec, np.float64)
    if grad_len is not None:
        gl = np.asarray(grad_len, np.float64)
        safe = np.where(length > 0.0, length, 1.0)
        g += np.where(length > 0.0, gl / safe, 0.0)[:, None] * v
    s = _structure_of(batch_ptr, src)
    Ls = lattices[s]
    gx = np.einsum("em,ekm->ek", g, Ls)            # g L^T
    grad_frac = np.zeros_like(frac)
    np.add.at(grad_frac, dst, gx)
    np.add.at(grad_frac, src, -gx)
    f = _frac_displacement(frac, src, dst, image)
    grad_lattice = np.zeros_like(lattices)
    np.add.at(grad_lattice, s, f[:, :, None] * g[:, None, :])
    return grad_frac, grad_lattice


def _objective(lattices, frac, batch_ptr, src, dst, image, gv, gl, edges):
    if edges.shape[0] == 0:
        return 0.0
    v, length = edge_geometry64(lattices, frac, batch_ptr, src[edges], dst[edges], image[edges])
    J = 0.0
    if gv is not None:
        J += float((gv[edges] * v).sum())
    if gl is not None:
        J += float((gl[edges] * length).sum())
    return J


def fd_vjp64(lattices, frac, batch_ptr, src, dst, image, grad_vec=None, grad_len=None,
             h: float = 1e-6, atoms=None, structures=None):
    """Central finite differences (step h, FP64) of J = sum_e g_v,e . v_e + g_l,e l_e.

    Only the edges that touch the perturbed atom (or structure) are re-evaluated.
    ``atoms`` / ``structures`` restrict which rows are probed (others stay NaN).
    Returns (grad_frac [N,3], grad_lattice [B,3,3]).
    """
    lattices = np.array(lattices, np.float64)
    frac = np.array(frac, np.float64)
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    image = np.asarray(image, np.int64).reshape(-1, 3)
    gv = None if grad_vec is None else np.asarray(grad_vec, np.float64)
    gl = None if grad_len is None else np.asarray(grad_len, np.float64)
    N, B = frac.shape[0], lattices.shape[0]
    s_of_edge = _structure_of(batch_ptr, src)
    gf = np.full((N, 3), np.nan)
    gL = np.full((B, 3, 3), np.nan)
    atoms = range(N) if atoms is None else atoms
    structures = range(B) if structures is None else structures
    for a in atoms:
        edges = np.nonzero((src == a) | (dst == a))[0]
        for c in range(3):
            old = frac[a, c]
            frac[a, c] = old + h
            jp = _objective(lattices, frac, batch_ptr, src, dst, image, gv, gl, edges)
            frac[a, c] = old - h
            jm = _objective(lattices, frac, batch_ptr, src, dst, image, gv, gl, edges)
            frac[a, c] = old
            gf[a, c] = (jp - jm) / (2.0 * h)
    for b in structures:
        edges = np.nonzero(s_of_edge == b)[0]
        for r in range(3):
            for c in range(3):
                old = lattices[b, r, c]
                lattices[b, r, c] = old + h
                jp = _objective(lattices, frac, batch_ptr, src, dst, image, gv, gl, edges)
                lattices[b, r, c] = old - h
                jm = _objective(lattices, frac, batch_ptr, src, dst, image, gv, gl, edges)
                lattices[b, r, c] = old
                gL[b, r, c] = (jp - jm) / (2.0 * h)
    return gf, gL


def gaussian_loss64(length, w, mu: float = 3.0) -> float:
    """sum_e w_e exp(-(l_e - mu)^2), the differentiation workload's loss."""
    length = np.asarray(length, np.float64)
    return float((np.asarray(w, np.float64) * np.exp(-(length - mu) ** 2)).sum())


def gaussian_loss_grad_len64(length, w, mu: float = 3.0) -> np.ndarray:
    """d loss / d l_e = -2 w_e (l_e - mu) exp(-(l_e - mu)^2)."""
    length = np.asarray(length, np.float64)
    w = np.asarray(w, np.float64)
    return -2.0 * w * (length - mu) * np.exp(-(length - mu) ** 2)
