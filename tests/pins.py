"""Pins for the FP64 oracle: checks against values fixed by the paper and by
mathematics (closed forms, invariants, brute force, finite differences).

Every check is a plain function taking the oracle package, so the same checks
run against the real oracle (``test_oracle_pins.py``) and against oracles with
a planted mistake (``test_oracle_mutations.py``), where at least one of them
must fail.
"""
from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _edges_set(src, dst, img):
    return {(int(a), int(b), int(t[0]), int(t[1]), int(t[2])) for a, b, t in zip(src, dst, img)}


# ----------------------------------------------------------------- closed forms


def pin_cubic_shells(O):
    """Neighbour counts of sc / bcc / fcc (conventional and primitive cells)."""
    g = golden("cubic_shells.json")
    for name in ("sc", "bcc", "fcc"):
        x = np.array(g[name]["frac"], np.float64)
        for c, want in zip(g[name]["cutoffs"], g[name]["edges_per_atom"]):
            src, dst, img, ln = O.cutoff_structure64(np.eye(3), x, c)
            counts = np.bincount(src, minlength=len(x))
            assert (counts == want).all(), (name, c, counts, want)
            assert (ln < c).all()
    for name in ("fcc_primitive", "bcc_primitive"):
        L = np.array(g[name]["lattice"], np.float64)
        for c, want in zip(g[name]["cutoffs"], g[name]["edges_per_atom"]):
            src, dst, img, ln = O.cutoff_structure64(L, np.zeros((1, 3)), c)
            assert len(src) == want, (name, c, len(src), want)


def pin_sc_sum_of_three_squares(O):
    """sc with a = 1: edges(c) = sum_{1 <= m < c^2} r3(m); shell lengths are sqrt(m)."""
    r3 = golden("cubic_shells.json")["r3"]["values"]
    for m_max in range(1, len(r3)):
        c = math.sqrt(m_max + 0.5)
        src, dst, img, ln = O.cutoff_structure64(np.eye(3), np.zeros((1, 3)), c)
        want = sum(r3[:m_max])
        assert len(src) == want, (c, len(src), want)
        sq = np.rint(ln * ln).astype(np.int64)
        assert np.allclose(ln * ln, sq, atol=1e-9)
        for m in range(1, m_max + 1):
            assert int((sq == m).sum()) == r3[m - 1], (m, int((sq == m).sum()), r3[m - 1])


def pin_strict_cutoff(O):
    """Definition def6 uses a strict '<': sc with a = 1 and c = 1 has no edge."""
    src, _, _, _ = O.cutoff_structure64(np.eye(3), np.zeros((1, 3)), 1.0)
    assert len(src) == 0
    src, _, _, _ = O.cutoff_structure64(2.0 * np.eye(3), np.zeros((1, 3)), 2.0)
    assert len(src) == 0


def pin_row_convention(O):
    """Rows of L are the lattice vectors: with rows (2,0,0), (1,2,0), (0,0,3) the
    image t = (0,1,0) of a single atom lies at (1,2,0), length sqrt(5)."""
    L = np.array([[2.0, 0, 0], [1.0, 2.0, 0], [0, 0, 3.0]])
    x = np.zeros((1, 3))
    src, dst, img, ln = O.cutoff_structure64(L, x, 2.1)
    assert _edges_set(src, dst, img) == {(0, 0, 1, 0, 0), (0, 0, -1, 0, 0)}
    src, dst, img, ln = O.cutoff_structure64(L, x, 2.3)
    want = {(0, 0, 1, 0, 0), (0, 0, -1, 0, 0), (0, 0, 0, 1, 0), (0, 0, 0, -1, 0),
            (0, 0, 1, -1, 0), (0, 0, -1, 1, 0)}
    assert _edges_set(src, dst, img) == want
    v, l = O.edge_geometry64(L[None], x, np.array([0, 1]), np.array([0]), np.array([0]),
                             np.array([[0, 1, 0]]))
    assert np.allclose(v[0], [1.0, 2.0, 0.0], atol=1e-15) and abs(l[0] - math.sqrt(5)) < 1e-15


def pin_figure1(O):
    """Fig. 1: two atoms, edges carry the cell of the target."""
    g = golden("paper_figure1.json")
    L = np.array(g["lattice"])
    x = np.array(g["frac"])
    src, dst, img, ln = O.cutoff_structure64(L, x, g["cutoff"])
    want = {(0, 1) + tuple(t) for t in g["edges"]["0->1"]} | {(1, 0) + tuple(t) for t in g["edges"]["1->0"]}
    assert _edges_set(src, dst, img) == want
    assert np.allclose(ln, g["length"], atol=1e-15)
    v, l = O.edge_geometry64(L[None], x, np.array([0, 2]), src, dst, img)
    assert np.allclose(l, g["length"], atol=1e-15)
    assert np.allclose(np.abs(v), 0.5, atol=1e-15)


def pin_knn_tie_break(O):
    """sc, a = 1, k = 8: the six unit vectors then (-1,-1,0), (-1,0,-1)
    (key = (length, dst, t lexicographic ascending)); exact in FP64."""
    src, dst, img, ln, dk, _, _ = O.knn_structure64(np.eye(3), np.zeros((1, 3)), 8)
    want = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 1), (0, 1, 0), (1, 0, 0), (-1, -1, 0),
            (-1, 0, -1)]
    assert [tuple(int(a) for a in t) for t in img] == want
    assert np.allclose(ln, [1] * 6 + [math.sqrt(2)] * 2, atol=1e-15)
    # bcc, k = 10: 8 nearest at sqrt(3)/2 (all to the other atom), then 2 of the 6 at 1.
    x = np.array([[0, 0, 0], [0.5, 0.5, 0.5]])
    src, dst, img, ln, dk, _, _ = O.knn_structure64(np.eye(3), x, 10)
    assert (dst[:8] == 1).all() and (dst[10:18] == 0).all()
    assert [tuple(int(a) for a in t) for t in img[:8]] == [tuple(t) for t in itertools.product((-1, 0), repeat=3)]
    assert [tuple(int(a) for a in t) for t in img[8:10]] == [(-1, 0, 0), (0, -1, 0)]
    assert [tuple(int(a) for a in t) for t in img[10:18]] == [tuple(t) for t in itertools.product((0, 1), repeat=3)]
    assert np.allclose(dk, [1.0, 1.0], atol=1e-15)


def pin_knn_single_atom_and_cluster(O):
    """KNN of a one-atom cell uses only self images (k-th distance of sc = the
    k-th lattice shell), and a tight cluster in a big cell needs the search to
    extend beyond the density-based first radius."""
    src, dst, img, ln, dk, _, _ = O.knn_structure64(2.0 * np.eye(3), np.zeros((1, 3)), 26)
    assert (dst == 0).all() and np.allclose(dk, 2.0 * math.sqrt(3.0))
    x = np.array([[0.5, 0.5, 0.5], [0.51, 0.5, 0.5], [0.5, 0.51, 0.5], [0.5, 0.5, 0.51]])
    L = 10.0 * np.eye(3)
    src, dst, img, ln, dk, _, _ = O.knn_structure64(L, x, 5)
    # 3 in-cluster neighbours, then 2 images of the cluster one cell away
    assert np.allclose(ln.reshape(4, 5)[:, :3].max(axis=1), [0.1, math.sqrt(2) * 0.1,
                       math.sqrt(2) * 0.1, math.sqrt(2) * 0.1], atol=1e-9)
    assert (ln.reshape(4, 5)[:, 3:] > 9.8).all() and (ln.reshape(4, 5)[:, 3:] < 10.2).all()


# ------------------------------------------------------------------ invariants


def _random_structure(rng, n, lo=3.0, hi=9.0, min_vf=0.2):
    from paper_2307_05380_amd.inputs import cell_from_parameters, volume_factor
    while True:
        ang = np.deg2rad(rng.uniform(50, 130, 3))
        vf = volume_factor(*ang)
        if vf == vf and vf >= min_vf:
            break
    L = cell_from_parameters(*rng.uniform(lo, hi, 3), *ang)
    R = np.linalg.qr(rng.normal(size=(3, 3)))[0]      # arbitrary orientation
    return (L @ R).astype(np.float32).astype(np.float64), rng.random((n, 3)).astype(np.float32).astype(np.float64)


def pin_symmetry(O, seed=1):
    """(i, j, t) is an edge iff (j, i, -t) is, with the same length."""
    rng = np.random.default_rng(seed)
    for _ in range(4):
        L, x = _random_structure(rng, int(rng.integers(1, 7)))
        src, dst, img, ln = O.cutoff_structure64(L, x, 7.0)
        keys = [(int(a), int(b), int(t[0]), int(t[1]), int(t[2])) for a, b, t in zip(src, dst, img)]
        d = dict(zip(keys, ln))
        assert len(d) == len(src) > 0
        for (i, j, t0, t1, t2), l in d.items():
            r = (j, i, -t0, -t1, -t2)
            assert r in d, r
            assert abs(d[r] - l) < 1e-12


def pin_supercell(O, seed=2):
    """An m1 x m2 x m3 supercell has prod(m) times the edges and the exact image map
    (i_u -> j_{(u+t) mod m}, floor((u+t)/m)) of the primitive edges."""
    rng = np.random.default_rng(seed)
    L, x = _random_structure(rng, 3, 3.0, 6.0, 0.3)
    c = 6.5
    m = np.array([2, 1, 3])
    src, dst, img, ln = O.cutoff_structure64(L, x, c)
    cells = np.array(list(itertools.product(range(m[0]), range(m[1]), range(m[2]))))
    n = len(x)
    xs = ((cells[:, None, :] + x[None, :, :]) / m).reshape(-1, 3)
    Ls = L * m[:, None]
    s2, d2, i2, l2 = O.cutoff_structure64(Ls, xs, c)
    assert len(s2) == len(src) * int(m.prod())
    index = {tuple(u): a for a, u in enumerate(cells)}
    want = set()
    for a, u in enumerate(cells):
        for i, j, t in zip(src, dst, img):
            w = u + t
            want.add((a * n + int(i), index[tuple(np.mod(w, m))] * n + int(j)) + tuple(int(q) for q in np.floor_divide(w, m)))
    assert _edges_set(s2, d2, i2) == want
    # the same per-atom sorted lengths
    for a in range(len(cells)):
        for i in range(n):
            l_p = np.sort(ln[src == i])
            l_s = np.sort(l2[s2 == a * n + i])
            assert np.allclose(l_p, l_s, atol=1e-9)


def pin_unimodular(O, seed=3):
    """L' = U L and x' = x U^{-1} describe the same crystal: per-atom length
    multisets agree and t' = t U^{-1}."""
    rng = np.random.default_rng(seed)
    L, x = _random_structure(rng, 3, 4.0, 7.0, 0.4)
    U = np.array([[1, 1, 0], [0, 1, 0], [1, 0, 1]], np.float64)     # det 1
    Ui = np.linalg.inv(U)
    L2, x2 = U @ L, x @ Ui
    c = 6.0
    s1, d1, i1, l1 = O.cutoff_structure64(L, x, c)
    s2, d2, i2, l2 = O.cutoff_structure64(L2, x2, c)
    assert len(s1) == len(s2)
    mapped = {(int(a), int(b)) + tuple(int(q) for q in np.rint(t @ Ui)) for a, b, t in zip(s1, d1, i1)}
    assert mapped == _edges_set(s2, d2, i2)
    for i in range(len(x)):
        assert np.allclose(np.sort(l1[s1 == i]), np.sort(l2[s2 == i]), atol=1e-9)


def pin_translation(O, seed=4):
    """Shifting every atom by the same vector changes nothing."""
    rng = np.random.default_rng(seed)
    L, x = _random_structure(rng, 4)
    s1, d1, i1, l1 = O.cutoff_structure64(L, x, 6.0)
    s2, d2, i2, l2 = O.cutoff_structure64(L, x + np.array([0.25, -0.125, 0.5]), 6.0)
    assert _edges_set(s1, d1, i1) == _edges_set(s2, d2, i2)
    assert np.allclose(l1, l2, atol=1e-12)


def pin_enormous_range(O, seed=5):
    """Brute force over t in [-M, M]^3 with M far beyond any bound, on tiny cells
    including thin, strongly skewed ones; coordinates outside [0,1) too."""
    from paper_2307_05380_amd.inputs import cell_from_parameters
    rng = np.random.default_rng(seed)
    cells = [
        cell_from_parameters(2.5, 2.7, 3.1, *np.deg2rad([20.0, 20.0, 38.0])),    # volume factor 0.074
        cell_from_parameters(3.0, 2.5, 6.0, *np.deg2rad([150.0, 40.0, 130.0])),
        cell_from_parameters(2.5, 2.5, 2.5, *np.deg2rad([60.0, 60.0, 60.0])),
        np.array([[3.0, 0, 0], [2.9, 0.4, 0], [1.0, 1.0, 0.3]]),
    ]
    for L in cells:
        for n in (1, 2):
            x = rng.uniform(-0.7, 1.6, (n, 3))
            c = 4.0
            Li = np.linalg.inv(L)
            M = int(2 * np.ceil(c * np.sqrt((Li * Li).sum(0))).max() + 6)
            T = np.array(list(itertools.product(range(-M, M + 1), repeat=3)), np.float64)
            want = set()
            for i in range(n):
                for j in range(n):
                    v = (x[j] - x[i] + T) @ L
                    ln = np.sqrt((v * v).sum(1))
                    for t in T[ln < c]:
                        if i == j and not t.any():
                            continue
                        want.add((i, j) + tuple(int(q) for q in t))
            src, dst, img, ln = O.cutoff_structure64(L, x, c)
            assert _edges_set(src, dst, img) == want, (L, len(want), len(src))


def pin_knn_vs_cutoff(O, seed=6):
    """KNN edges lie inside the cutoff graph at c = d_k + 2e-4, and the k-th KNN
    length equals the k-th smallest cutoff length of the same source."""
    rng = np.random.default_rng(seed)
    for n, k in ((1, 12), (5, 8), (9, 16)):
        L, x = _random_structure(rng, n, 3.0, 8.0, 0.3)
        s, d, t, ln, dk, _, _ = O.knn_structure64(L, x, k)
        c = float(dk.max()) + 2e-4
        cs, cd, ct, cl = O.cutoff_structure64(L, x, c)
        assert _edges_set(s, d, t) <= _edges_set(cs, cd, ct)
        for i in range(n):
            li = np.sort(cl[cs == i])
            assert abs(li[k - 1] - dk[i]) < 1e-12
            assert np.allclose(ln[i * k:(i + 1) * k], li[:k], atol=1e-12)


# -------------------------------------------------------------------- gradients


def _grad_case(rng, O):
    Ls, xs = [], []
    for n in (2, 3):
        L, x = _random_structure(rng, n, 3.0, 5.0, 0.4)
        Ls.append(L)
        xs.append(x)
    lat = np.stack(Ls)
    frac = np.concatenate(xs)
    ptr = np.array([0, 2, 5])
    src, dst, img = [], [], []
    for b in range(2):
        s, d, t, _ = O.cutoff_structure64(lat[b], frac[ptr[b]:ptr[b + 1]], 4.5)
        src.append(s + ptr[b])
        dst.append(d + ptr[b])
        img.append(t)
    return lat, frac, ptr, np.concatenate(src), np.concatenate(dst), np.concatenate(img)


def pin_gradients(O, seed=7):
    """Analytic VJP against FP64 central differences, plus identities:
    sum_i grad_x[i] = 0 per structure (translation invariance), L^T G_L symmetric
    for a length-only loss (rotation invariance) and tr(L^T G_L) = sum_e l_e g_l,e
    (lengths are homogeneous of degree 1 in L)."""
    rng = np.random.default_rng(seed)
    lat, frac, ptr, src, dst, img = _grad_case(rng, O)
    E = len(src)
    gv = rng.normal(size=(E, 3))
    gl = rng.normal(size=E)
    for a, b in ((gv, gl), (gv, None), (None, gl)):
        gf, gL = O.edge_geometry_vjp64(lat, frac, ptr, src, dst, img, a, b)
        ff, fL = O.fd_vjp64(lat, frac, ptr, src, dst, img, a, b, h=1e-6)
        scale = max(np.abs(gf).max(), np.abs(gL).max())
        assert np.abs(gf - ff).max() <= 1e-6 * scale, np.abs(gf - ff).max()
        assert np.abs(gL - fL).max() <= 1e-6 * scale, np.abs(gL - fL).max()
        for s in range(2):
            assert np.abs(gf[ptr[s]:ptr[s + 1]].sum(0)).max() <= 1e-9 * scale
    gf, gL = O.edge_geometry_vjp64(lat, frac, ptr, src, dst, img, None, gl)
    _, ln = O.edge_geometry64(lat, frac, ptr, src, dst, img)
    s_of = np.searchsorted(ptr, src, side="right") - 1
    for s in range(2):
        M = lat[s].T @ gL[s]
        assert np.abs(M - M.T).max() <= 1e-9 * np.abs(M).max()
        assert abs(np.trace(M) - float((ln * gl)[s_of == s].sum())) <= 1e-9 * np.abs(M).max()


# ------------------------------------------------------------ per-atom cutoffs


def pin_radii_closed_form(O):
    """CsCl arrangement (cubic a = 1, A at 0, B at the body centre): A-B at
    sqrt(3)/2, A-A and B-B at 1. With c_A = 0.95 and c_B = 1.05 every A has the
    8 B around it and every B the 8 A plus its 6 B images: the graph is not
    symmetric, and an edge's cutoff is its source's."""
    x = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
    src, dst, img, ln = O.cutoff_structure64(np.eye(3), x, np.array([0.95, 1.05]))
    counts = np.bincount(src, minlength=2)
    assert counts.tolist() == [8, 14], counts
    assert (dst[src == 0] == 1).all()
    assert np.allclose(ln[src == 0], math.sqrt(3.0) / 2.0)
    assert (np.sort(ln[src == 1])[8:] > 0.999).all()
    src, _, _, _ = O.cutoff_structure64(np.eye(3), x, np.array([0.8, 0.9]))
    assert np.bincount(src, minlength=2).tolist() == [0, 8]


def pin_radii_restriction(O, seed=8):
    """Per-atom cutoffs: the out-edges of source i are exactly the constant-cutoff
    graph at c = c_i restricted to i; equal radii give the constant graph."""
    rng = np.random.default_rng(seed)
    L, x = _random_structure(rng, 5)
    radii = rng.uniform(2.0, 6.0, size=5)
    s, d, t, ln = O.cutoff_structure64(L, x, radii)
    got = _edges_set(s, d, t)
    want = set()
    for i in range(5):
        cs, cd, ct, cl = O.cutoff_structure64(L, x, float(radii[i]))
        m = cs == i
        want |= _edges_set(cs[m], cd[m], ct[m])
    assert got == want
    s1, d1, t1, l1 = O.cutoff_structure64(L, x, np.full(5, 4.5))
    s2, d2, t2, l2 = O.cutoff_structure64(L, x, 4.5)
    assert _edges_set(s1, d1, t1) == _edges_set(s2, d2, t2)


# --------------------------------------------------------------------- triplets


def pin_triplets_closed_form(O):
    """Tetragonal cell a = b = 1, c = 1.5, one atom, cutoff 1.45: the 8 edges are
    +-x, +-y and the 4 in-plane diagonals (+-1, +-1, 0). 56 ordered pairs; their
    angles follow from those 8 vectors written out here."""
    L = np.diag([1.0, 1.0, 1.5])
    src, dst, img, ln = O.cutoff_structure64(L, np.zeros((1, 3)), 1.45)
    assert len(src) == 8
    ptr = np.array([0, 8])
    e1, e2 = O.triplets64(ptr)
    assert len(e1) == 56 and (e1 != e2).all()
    assert len(set(zip(e1.tolist(), e2.tolist()))) == 56
    vec, _ = O.edge_geometry64(L[None], np.zeros((1, 3)), np.array([0, 1]), src, dst, img)
    cos = O.triplet_cos64(vec, e1, e2)
    known = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0],
                      [1, 1, 0], [1, -1, 0], [-1, 1, 0], [-1, -1, 0]], np.float64)
    want = []
    for p, q in itertools.permutations(range(8), 2):
        u, w = known[p], known[q]
        want.append(float(u @ w) / math.sqrt(float(u @ u) * float(w @ w)))
    assert np.allclose(np.sort(cos), np.sort(want), atol=1e-12)
    assert np.isclose(np.sort(cos)[0], -1.0) and np.isclose(np.sort(cos)[-1], 1.0 / math.sqrt(2.0))


def pin_triplets_brute_force(O, seed=9):
    """Random degrees (including 0 and 1): the pairs are exactly the ordered
    pairs of distinct edges of each source, sum_i d_i (d_i - 1) of them, in
    (source, first, second) order."""
    rng = np.random.default_rng(seed)
    deg = rng.integers(0, 7, size=12)
    deg[3] = 0
    deg[5] = 1
    ptr = np.concatenate([[0], np.cumsum(deg)])
    e1, e2 = O.triplets64(ptr)
    want = []
    for i in range(12):
        want += list(itertools.permutations(range(ptr[i], ptr[i + 1]), 2))
    assert list(zip(e1.tolist(), e2.tolist())) == sorted(want)
    assert len(e1) == int((deg * (deg - 1)).sum())


# ------------------------------------------------------------- symmetrisation


def pin_symmetrize_chain(O):
    """Atoms at x = 0, 1, 3 (Angstrom) on a line in a 100 A cubic cell, k = 1:
    0 -> 1, 1 -> 0, 2 -> 1. The closure adds 1 -> 2 only, after 1's own edge."""
    L = 100.0 * np.eye(3)
    x = np.array([[0.0, 0, 0], [0.01, 0, 0], [0.03, 0, 0]])
    src, dst, img, ln, dk, near, inside = O.knn_structure64(L, x, 1)
    assert dst.tolist() == [1, 0, 1]
    ptr = np.arange(4, dtype=np.int64)
    sp, ss, sd, si, sl = O.symmetrize64(ptr, dst, img, ln)
    assert sp.tolist() == [0, 1, 3, 4]
    assert ss.tolist() == [0, 1, 1, 2] and sd.tolist() == [1, 0, 2, 1]
    assert np.allclose(sl, [1.0, 1.0, 2.0, 2.0])


def pin_symmetrize_properties(O, seed=10):
    """KNN graph of a random cell (k = 5, self images allowed): the closure is
    symmetric, equals E union reverse(E) as a set, keeps every source's own
    edges first and in order, and adds nothing when applied again; a cutoff
    graph (already symmetric) is returned unchanged."""
    rng = np.random.default_rng(seed)
    L, x = _random_structure(rng, 7)
    src, dst, img, ln, dk, near, inside = O.knn_structure64(L, x, 5)
    ptr = np.arange(0, 7 * 5 + 1, 5, dtype=np.int64)
    sp, ss, sd, si, sl = O.symmetrize64(ptr, dst, img, ln)
    S = _edges_set(ss, sd, si)
    E = _edges_set(src, dst, img)
    R = {(b, a, -t0, -t1, -t2) for a, b, t0, t1, t2 in E}
    assert S == E | R and len(S) == len(ss)
    assert all((b, a, -t0, -t1, -t2) in S for a, b, t0, t1, t2 in S)
    for i in range(7):
        assert np.array_equal(sd[sp[i]:sp[i] + 5], dst[5 * i:5 * i + 5])
    assert np.allclose(O.edge_geometry64(L[None], x, np.array([0, 7]), ss, sd, si)[1], sl, atol=1e-12)
    sp2, ss2, sd2, si2, _ = O.symmetrize64(sp, sd, si)
    assert np.array_equal(sp2, sp) and np.array_equal(sd2, sd) and np.array_equal(si2, si)
    cs, cd, ct, cl = O.cutoff_structure64(L, x, 4.0)
    cptr = np.concatenate([[0], np.cumsum(np.bincount(cs, minlength=7))])
    qp, qs, qd, qi, _ = O.symmetrize64(cptr, cd, ct)
    assert np.array_equal(qp, cptr) and np.array_equal(qd, cd) and np.array_equal(qi, ct)


# ------------------------------------------------------------ KNN with ties


def pin_knn_ties_shells(O):
    """Keeping ties returns whole coordination shells: sc (a = 1) with k = 4
    gives the 6 nearest, k = 7 gives 6 + 12 = 18; bcc (conventional, a = 1)
    with k = 3 gives 8; fcc with k = 13 gives 12 + 6 = 18."""
    g = golden("cubic_shells.json")
    one = np.zeros((1, 3))
    for k, want in ((4, 6), (7, 18), (1, 6), (6, 6)):
        s, d, t, ln, ptr = O.knn_ties_structure64(np.eye(3), one, k)
        assert len(s) == want and ptr.tolist() == [0, want], (k, len(s))
    bcc = np.array(g["bcc"]["frac"], np.float64)
    s, d, t, ln, ptr = O.knn_ties_structure64(np.eye(3), bcc, 3)
    assert np.diff(ptr).tolist() == [8] * len(bcc)
    fcc = np.array(g["fcc"]["frac"], np.float64)
    s, d, t, ln, ptr = O.knn_ties_structure64(np.eye(3), fcc, 13)
    assert np.diff(ptr).tolist() == [18] * len(fcc)
    assert np.allclose(np.sort(ln[:18]), [math.sqrt(0.5)] * 12 + [1.0] * 6)


def pin_knn_ties_generic(O, seed=11):
    """Without ties (random coordinates) the selection is exactly the KNN graph,
    in the same key order."""
    rng = np.random.default_rng(seed)
    L, x = _random_structure(rng, 6)
    s, d, t, ln, ptr = O.knn_ties_structure64(L, x, 5)
    ks, kd, kt, kl, dk, near, inside = O.knn_structure64(L, x, 5)
    assert np.array_equal(ptr, np.arange(0, 31, 5))
    assert np.array_equal(d, kd) and np.array_equal(t, kt) and np.allclose(ln, kl)


# ------------------------------------------------------ differentiation loss


def pin_gaussian_loss(O):
    """The differentiation workload's loss sum_e w_e exp(-(l_e - mu)^2) and its
    length gradient: closed values at l = mu (loss sum w, gradient 0), at
    l = mu + 1 (w / e) and at the gradient's extrema l = mu -+ 1/sqrt(2)
    (gradient -+ sqrt(2) w e^{-1/2}), and an FP64 central difference of the
    loss against the gradient at random lengths."""
    mu = 3.0
    w = np.array([0.7, -1.3, 2.0])
    at = np.full(3, mu)
    assert abs(O.gaussian_loss64(at, w, mu) - w.sum()) <= 1e-15 * 4
    assert np.abs(O.gaussian_loss_grad_len64(at, w, mu)).max() == 0.0
    assert abs(O.gaussian_loss64(at + 1.0, w, mu) - w.sum() / math.e) <= 1e-14
    s = 1.0 / math.sqrt(2.0)
    peak = math.sqrt(2.0) * math.exp(-0.5)
    assert np.allclose(O.gaussian_loss_grad_len64(at - s, w, mu), peak * w, rtol=1e-14, atol=0)
    assert np.allclose(O.gaussian_loss_grad_len64(at + s, w, mu), -peak * w, rtol=1e-14, atol=0)
    rng = np.random.default_rng(12)
    ln = rng.uniform(0.5, 6.0, size=40)
    wr = rng.standard_normal(40)
    g = O.gaussian_loss_grad_len64(ln, wr, mu)
    h = 1e-6
    for e in range(len(ln)):
        up, dn = ln.copy(), ln.copy()
        up[e] += h
        dn[e] -= h
        fd = (O.gaussian_loss64(up, wr, mu) - O.gaussian_loss64(dn, wr, mu)) / (2 * h)
        assert abs(fd - g[e]) <= 1e-7 * max(1.0, abs(g[e])), (e, fd, g[e])


ALL_PINS = [pin_cubic_shells, pin_sc_sum_of_three_squares, pin_strict_cutoff, pin_row_convention,
            pin_figure1, pin_knn_tie_break, pin_knn_single_atom_and_cluster, pin_symmetry,
            pin_supercell, pin_unimodular, pin_translation, pin_enormous_range, pin_knn_vs_cutoff,
            pin_gradients, pin_radii_closed_form, pin_radii_restriction, pin_triplets_closed_form,
            pin_triplets_brute_force, pin_symmetrize_chain, pin_symmetrize_properties,
            pin_knn_ties_shells, pin_knn_ties_generic, pin_gaussian_loss]
