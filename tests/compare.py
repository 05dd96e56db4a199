"""GPU-vs-oracle comparison rules (test side).

Edge sets must match the FP64 oracle exactly, except for candidates whose FP64
length lies within BAND of the cutoff (cutoff graphs) or of the k-th distance
(KNN graphs): those are counted, not judged. Edge lengths must agree with the
FP64 length of the same edge within LEN_TOL. Both tolerances are the ones
fixed for this method's FP32 sweep (1e-4 A band, 2e-5 A lengths).
"""
from __future__ import annotations

import numpy as np

import oracle

BAND = 1e-4
LEN_TOL = 2e-5


def _rows(src, dst, img):
    a = np.empty((len(src), 5), np.int64)
    a[:, 0] = src
    a[:, 1] = dst
    a[:, 2:] = np.asarray(img).reshape(-1, 3)
    return a


def _void(a):
    a = np.ascontiguousarray(a, np.int64)
    return a.view(np.dtype((np.void, a.dtype.itemsize * a.shape[1]))).ravel()


def _cut_of(radii, cutoff, src):
    """The cutoff of every edge: its source's radius, or the constant."""
    if radii is None:
        return np.full(len(src), float(cutoff))
    return np.asarray(radii, np.float64)[np.asarray(src, np.int64)]


def cutoff_check(batch, g_src, g_dst, g_img, g_len, structures=None, band=BAND, len_tol=LEN_TOL,
                 processes=None, radii=None):
    """Compare GPU cutoff edges (numpy, global indices) with the oracle on the
    given structures (``radii``: optional per-atom cutoffs [N], float32 values
    as given to the GPU). Returns a stats dict; raises AssertionError on mismatch."""
    ptr = batch.batch_ptr
    if structures is None:
        structures = list(range(batch.B))
    structures = [int(s) for s in structures]
    cut = batch.cutoff if radii is None else np.asarray(radii, np.float32).astype(np.float64)
    og = oracle.cutoff_graph64(batch.lattices, batch.frac, ptr, cut, band=band,
                               structures=structures, processes=processes)
    # GPU edges of the selected structures
    s_of_src = np.searchsorted(ptr, g_src, side="right") - 1
    sel = np.isin(s_of_src, np.asarray(structures))
    G = _rows(g_src[sel], g_dst[sel], g_img[sel])
    GL = np.asarray(g_len)[sel].astype(np.float64)
    O = _rows(og.src, og.dst, og.image)
    OL = og.length
    gv, ov = _void(G), _void(O)
    assert np.unique(gv).shape[0] == gv.shape[0], "duplicate GPU edges"
    c = _cut_of(radii, batch.cutoff, og.src)
    cg = _cut_of(None if radii is None else np.asarray(radii, np.float32), batch.cutoff, G[:, 0])
    must = OL < c - band
    near = np.abs(OL - c) <= band
    in_o = np.isin(gv, ov)
    assert in_o.all(), f"{int((~in_o).sum())} GPU edges are not edges of the oracle (first: {G[~in_o][:3]})"
    found = np.isin(ov[must], gv)
    assert found.all(), f"{int((~found).sum())} oracle edges missing on GPU (first: {O[must][~found][:3]})"
    # lengths of matched edges
    order_o = np.argsort(ov)
    pos = order_o[np.searchsorted(ov[order_o], gv)]
    err = np.abs(GL - OL[pos])
    assert err.max(initial=0.0) <= len_tol, f"length error {err.max():.3g} > {len_tol}"
    # the strict cutoff holds in the GPU's own precision (FP32 length vs FP32 cutoff)
    assert (np.asarray(g_len)[sel] < cg.astype(np.float32)).all()
    return {"edges": int(G.shape[0]), "oracle_inside": int(must.sum()), "near": int(near.sum()),
            "near_on_gpu": int(np.isin(ov[near], gv).sum()), "max_len_err": float(err.max(initial=0.0))}


def knn_check(batch, k, g_src, g_dst, g_img, g_len, sources=None, band=BAND, len_tol=LEN_TOL,
              processes=None):
    """Compare GPU KNN edges ([N*k], source-major) with the oracle on the given
    structures' sources (or all). Returns stats; raises AssertionError on mismatch."""
    ptr = batch.batch_ptr
    structures = sorted(set(int(s) for s in (sources if sources is not None else range(batch.B))))
    ok = oracle.knn_graph64(batch.lattices, batch.frac, ptr, k, band=band, structures=structures,
                            processes=processes)
    g_src = np.asarray(g_src).reshape(-1, k)
    g_dst = np.asarray(g_dst).reshape(-1, k)
    g_img = np.asarray(g_img).reshape(-1, k, 3)
    g_len = np.asarray(g_len).reshape(-1, k).astype(np.float64)
    atoms = np.concatenate([np.arange(ptr[s], ptr[s + 1]) for s in structures]) if structures else np.zeros(0, np.int64)
    o_dst = ok.graph.dst.reshape(-1, k)
    o_img = ok.graph.image.reshape(-1, k, 3)
    o_len = ok.graph.length.reshape(-1, k)
    near_total = 0
    # FP64 lengths of the GPU's own edges
    gs = np.repeat(atoms, k)
    gd = g_dst[atoms].ravel()
    gi = g_img[atoms].reshape(-1, 3)
    assert (gd >= 0).all(), "GPU wrote invalid KNN edges"
    _, l64 = oracle.edge_geometry64(batch.lattices, batch.frac, ptr, gs, gd, gi)
    l64 = l64.reshape(-1, k)
    assert (np.abs(l64 - g_len[atoms]) <= len_tol).all(), \
        f"length error {np.abs(l64 - g_len[atoms]).max():.3g}"
    for r, a in enumerate(atoms):
        assert (g_src[a] == a).all()
        dk = ok.dk[r]
        gset = {(int(d),) + tuple(int(q) for q in t) for d, t in zip(g_dst[a], g_img[a])}
        assert len(gset) == k, f"source {a}: duplicate edges"
        assert (int(a), 0, 0, 0) not in gset, f"source {a}: self image selected"
        inside = {(int(d),) + tuple(int(q) for q in t)
                  for d, t, l in zip(o_dst[r], o_img[r], o_len[r]) if l < dk - band}
        missing = inside - gset
        assert not missing, f"source {a}: oracle neighbours missing {sorted(missing)[:3]}"
        assert (l64[r] <= dk + band).all(), f"source {a}: selected beyond the k-th distance"
        # the GPU's own order: (length32, dst, t) ascending
        keys = list(zip(g_len[a], g_dst[a], g_img[a][:, 0], g_img[a][:, 1], g_img[a][:, 2]))
        assert keys == sorted(keys), f"source {a}: not in (length, dst, t) order"
        near_total += len(ok.near.get(int(a), []))
    return {"sources": int(len(atoms)), "near": int(near_total),
            "max_len_err": float(np.abs(l64 - g_len[atoms]).max(initial=0.0))}


def cutoff_sources_check(batch, s, sources, g_src, g_dst, g_img, g_len, band=BAND, len_tol=LEN_TOL,
                         radii=None):
    """cutoff_check restricted to some sources (local indices) of structure s."""
    a0 = int(batch.batch_ptr[s])
    L, x = batch.structure(s)
    a1 = int(batch.batch_ptr[s + 1])
    cut = batch.cutoff if radii is None else np.asarray(radii, np.float32)[a0:a1].astype(np.float64)
    os_, od, oi, ol = oracle.cutoff_sources64(L, x, cut, sources, band=band)
    glob = a0 + np.asarray(sources, np.int64)
    sel = np.isin(g_src, glob)
    G = _rows(g_src[sel], g_dst[sel], g_img[sel])
    GL = np.asarray(g_len)[sel].astype(np.float64)
    O = _rows(os_ + a0, od + a0, oi)
    gv, ov = _void(G), _void(O)
    assert np.unique(gv).shape[0] == gv.shape[0], "duplicate GPU edges"
    c = _cut_of(None if radii is None else np.asarray(radii, np.float64)[a0:a1], batch.cutoff, os_)
    must = ol < c - band
    in_o = np.isin(gv, ov)
    assert in_o.all(), f"{int((~in_o).sum())} GPU edges are not edges of the oracle (first: {G[~in_o][:3]})"
    found = np.isin(ov[must], gv)
    assert found.all(), f"{int((~found).sum())} oracle edges missing on GPU (first: {O[must][~found][:3]})"
    order_o = np.argsort(ov)
    pos = order_o[np.searchsorted(ov[order_o], gv)]
    err = np.abs(GL - ol[pos])
    assert err.max(initial=0.0) <= len_tol, f"length error {err.max():.3g}"
    return {"edges": int(G.shape[0]), "near": int((np.abs(ol - c) <= band).sum()),
            "max_len_err": float(err.max(initial=0.0))}


def knn_sources_check(batch, s, k, sources, g_src, g_dst, g_img, g_len, band=BAND, len_tol=LEN_TOL):
    """knn_check restricted to some sources (local indices) of structure s."""
    a0 = int(batch.batch_ptr[s])
    L, x = batch.structure(s)
    src, dst, img, ln, dk, near, inside = oracle.knn_structure64(L, x, k, band=band, sources=sources)
    g_dst = np.asarray(g_dst).reshape(-1, k)
    g_img = np.asarray(g_img).reshape(-1, k, 3)
    g_len = np.asarray(g_len).reshape(-1, k).astype(np.float64)
    for r, il in enumerate(sources):
        a = a0 + int(il)
        assert (g_dst[a] >= 0).all(), f"source {a}: invalid edges"
        gset = {(int(d),) + tuple(int(q) for q in t) for d, t in zip(g_dst[a], g_img[a])}
        assert len(gset) == k and (a, 0, 0, 0) not in gset
        want = {(int(d) + a0,) + tuple(int(q) for q in t)
                for d, t, l in zip(dst[r * k:(r + 1) * k], img[r * k:(r + 1) * k], ln[r * k:(r + 1) * k])
                if l < dk[r] - band}
        assert not (want - gset), f"source {a}: missing {sorted(want - gset)[:3]}"
        gs = np.full(k, a)
        _, l64 = oracle.edge_geometry64(batch.lattices, batch.frac, batch.batch_ptr, gs, g_dst[a], g_img[a])
        assert (l64 <= dk[r] + band).all(), f"source {a}: beyond the k-th distance"
        assert np.abs(l64 - g_len[a]).max() <= len_tol
        keys = list(zip(g_len[a], g_dst[a], g_img[a][:, 0], g_img[a][:, 1], g_img[a][:, 2]))
        assert keys == sorted(keys), f"source {a}: not in (length, dst, t) order"
    return {"sources": len(sources)}
