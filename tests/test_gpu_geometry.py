"""Edge geometry forward / backward on the GPU against the FP64 oracle."""
import numpy as np
import pytest
import torch

import gpu_util as gu
import oracle
from paper_2307_05380_amd import _lib, graph, inputs

pytestmark = pytest.mark.gpu


def _edges(b):
    g = gu.cutoff(b)
    return g, gu.np_graph(g)


def test_forward_parity_config4():
    b = inputs.make_config(4)
    g, (s, d, t, ln) = _edges(b)
    L, X, P = gu.dev(b)
    vec, length = graph.edge_geometry(L, X, P, g.src, g.dst, g.image)
    v64, l64 = oracle.edge_geometry64(b.lattices, b.frac, b.batch_ptr, s, d, t)
    assert np.abs(vec.detach().cpu().numpy() - v64).max() <= 2e-5
    assert np.abs(length.detach().cpu().numpy() - l64).max() <= 2e-5
    # the graph's own lengths agree with the geometry op
    assert np.abs(length.detach().cpu().numpy() - ln).max() <= 2e-5


@pytest.mark.parametrize("order", ["shuffled", "structures_reversed", "cross_and_invalid"])
def test_forward_edge_orders(order):
    """The forward pass for edges that are not in the builders' order: fully
    shuffled, structure blocks reversed, or the builders' order with one edge
    whose dst lies in another structure and two edges with an endpoint outside
    [0, N) (those give NaN). Valid edges must match the oracle (the lattice of
    the source's structure)."""
    rng = np.random.default_rng(91)
    b = inputs.random_batch(rng, 10, 3, 60, 3.0, 8.0, cutoff=5.0)
    g, (s, d, t, ln) = _edges(b)
    s, d, t = s.astype(np.int64), d.astype(np.int64), t.copy()
    bad = np.zeros(len(s), bool)
    if order == "shuffled":
        perm = rng.permutation(len(s))
        s, d, t = s[perm], d[perm], t[perm]
    elif order == "structures_reversed":
        blocks = [np.flatnonzero((s >= b.batch_ptr[q]) & (s < b.batch_ptr[q + 1])) for q in range(b.B)]
        perm = np.concatenate(blocks[::-1])
        s, d, t = s[perm], d[perm], t[perm]
    else:
        q5 = int(np.searchsorted(b.batch_ptr, s[5], side="right")) - 1
        other_q = next(q for q in range(q5 + 1, q5 + b.B) if b.batch_ptr[q % b.B + 1] > b.batch_ptr[q % b.B]) % b.B
        d[5] = b.batch_ptr[other_q]                      # an atom of another structure
        s[10] = -1
        d[20] = b.N
        bad[[10, 20]] = True
    L, X, P = gu.dev(b)
    ti = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.int32))).cuda()
    vec, length = graph.edge_geometry(L, X, P, ti(s), ti(d), ti(t))
    vec, length = vec.detach().cpu().numpy(), length.detach().cpu().numpy()
    ok = ~bad
    v64, l64 = oracle.edge_geometry64(b.lattices, b.frac, b.batch_ptr, s[ok], d[ok], t[ok])
    assert np.abs(vec[ok] - v64).max() <= 2e-5
    assert np.abs(length[ok] - l64).max() <= 2e-5
    assert np.isnan(vec[bad]).all() and np.isnan(length[bad]).all()


def _rel_err(a, ref):
    return np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-300)


def test_backward_parity_config4_loss():
    """Loss = sum_e w_e exp(-(l_e - 3)^2), w_e ~ N(0,1) in canonical edge order;
    gradients to frac [N,3] and lattice [B,3,3] against the oracle's analytic
    gradient at 1e-4 relative, per structure and tensor."""
    b = inputs.make_config(4)
    g, (s, d, t, ln) = _edges(b)
    order = np.lexsort((t[:, 2], t[:, 1], t[:, 0], d, s))
    w = np.empty(len(s), np.float32)
    w[order] = inputs.loss_weights(len(s))
    L, X, P = gu.dev(b)
    L.requires_grad_(True)
    X.requires_grad_(True)
    vec, length = graph.edge_geometry(L, X, P, g.src, g.dst, g.image)
    wt = torch.from_numpy(w).cuda()
    loss = (wt * torch.exp(-(length - 3.0) ** 2)).sum()
    loss.backward()
    gl64 = oracle.gaussian_loss_grad_len64(oracle.edge_geometry64(b.lattices, b.frac, b.batch_ptr, s, d, t)[1], w)
    gf64, gL64 = oracle.edge_geometry_vjp64(b.lattices, b.frac, b.batch_ptr, s, d, t, None, gl64)
    gf = X.grad.cpu().numpy()
    gL = L.grad.cpu().numpy()
    worst_f = worst_L = 0.0
    for q in range(b.B):
        a0, a1 = b.batch_ptr[q], b.batch_ptr[q + 1]
        if np.abs(gf64[a0:a1]).max() > 0:
            worst_f = max(worst_f, _rel_err(gf[a0:a1], gf64[a0:a1]))
        if np.abs(gL64[q]).max() > 0:
            worst_L = max(worst_L, _rel_err(gL[q], gL64[q]))
    print("worst relative errors", worst_f, worst_L)
    assert worst_f <= 1e-4 and worst_L <= 1e-4


def test_backward_vs_finite_differences():
    rng = np.random.default_rng(4)
    b = inputs.random_batch(rng, 3, 2, 6, 3.0, 6.0, cutoff=4.5)
    g, (s, d, t, ln) = _edges(b)
    E = len(s)
    gv = rng.normal(size=(E, 3)).astype(np.float32)
    glen = rng.normal(size=E).astype(np.float32)
    L, X, P = gu.dev(b)
    run = graph.GeometryRunner(b.B, b.N)
    gf = torch.empty_like(X)
    gL = torch.empty_like(L)
    run.backward(L, X, P, g.src, g.dst, g.image, torch.from_numpy(gv).cuda(), torch.from_numpy(glen).cuda(), gf, gL)
    ff, fL = oracle.fd_vjp64(b.lattices, b.frac, b.batch_ptr, s, d, t, gv, glen, h=1e-6)
    assert _rel_err(gf.cpu().numpy(), ff) <= 1e-4
    assert _rel_err(gL.cpu().numpy(), fL) <= 1e-4
    # sum of coordinate gradients of a structure vanishes
    for q in range(b.B):
        a0, a1 = b.batch_ptr[q], b.batch_ptr[q + 1]
        assert np.abs(gf.cpu().numpy()[a0:a1].sum(0)).max() <= 1e-4 * np.abs(ff).max()


def test_backward_random_edge_order():
    """Edges in arbitrary order (no grouping by source) and only grad_vec."""
    rng = np.random.default_rng(8)
    b = inputs.random_batch(rng, 5, 3, 40, 3.0, 8.0, cutoff=5.0)
    g, (s, d, t, ln) = _edges(b)
    perm = rng.permutation(len(s))
    s, d, t = s[perm], d[perm], t[perm]
    gv = rng.normal(size=(len(s), 3)).astype(np.float32)
    L, X, P = gu.dev(b)
    run = graph.GeometryRunner(b.B, b.N)
    gf = torch.empty_like(X)
    gL = torch.empty_like(L)
    ti = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.int32))).cuda()
    run.backward(L, X, P, ti(s), ti(d), ti(t), torch.from_numpy(gv).cuda(), None, gf, gL)
    rf, rL = oracle.edge_geometry_vjp64(b.lattices, b.frac, b.batch_ptr, s, d, t, gv, None)
    assert _rel_err(gf.cpu().numpy(), rf) <= 1e-4
    assert _rel_err(gL.cpu().numpy(), rL) <= 1e-4


@pytest.mark.parametrize("order", ["structures_reversed", "shuffled_in_structure", "reversed_in_structure"])
def test_backward_partial_orders(order):
    """Edge orders that are grouped in some ways but not others: structure
    blocks in reverse order (each sorted by source), each structure's edges
    shuffled, or each structure's edges reversed. The result must not depend
    on the order."""
    rng = np.random.default_rng(81)
    b = inputs.random_batch(rng, 12, 3, 60, 3.0, 8.0, cutoff=5.0)
    g, (s, d, t, ln) = _edges(b)
    blocks = [np.flatnonzero((s >= b.batch_ptr[q]) & (s < b.batch_ptr[q + 1])) for q in range(b.B)]
    if order == "structures_reversed":
        perm = np.concatenate(blocks[::-1])
    elif order == "shuffled_in_structure":
        perm = np.concatenate([rng.permutation(x) for x in blocks])
    else:
        perm = np.concatenate([x[::-1] for x in blocks])
    assert len(perm) == len(s)
    s, d, t = s[perm], d[perm], t[perm]
    gv = rng.normal(size=(len(s), 3)).astype(np.float32)
    glen = rng.normal(size=len(s)).astype(np.float32)
    L, X, P = gu.dev(b)
    run = graph.GeometryRunner(b.B, b.N)
    gf = torch.empty_like(X)
    gL = torch.empty_like(L)
    ti = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.int32))).cuda()
    run.backward(L, X, P, ti(s), ti(d), ti(t), torch.from_numpy(gv).cuda(), torch.from_numpy(glen).cuda(), gf, gL)
    rf, rL = oracle.edge_geometry_vjp64(b.lattices, b.frac, b.batch_ptr, s, d, t, gv, glen)
    _per_structure_check(b, gf.cpu().numpy(), gL.cpu().numpy(), rf, rL)


def _per_structure_check(b, gf, gL, rf, rL, tol=1e-4):
    worst_f = worst_L = 0.0
    for q in range(b.B):
        a0, a1 = b.batch_ptr[q], b.batch_ptr[q + 1]
        if np.abs(rf[a0:a1]).max() > 0:
            worst_f = max(worst_f, _rel_err(gf[a0:a1], rf[a0:a1]))
        if np.abs(rL[q]).max() > 0:
            worst_L = max(worst_L, _rel_err(gL[q], rL[q]))
    print("worst relative errors", worst_f, worst_L)
    assert worst_f <= tol and worst_L <= tol


@pytest.mark.parametrize("m", [6, 8])
@pytest.mark.parametrize("buckets", [True, False])
def test_backward_supercells(m, buckets):
    """Structures large enough that one structure's edges are split over
    several workgroups (m = 6: 1728 atoms, ~10^5 edges) or exceed the LDS
    atom window (m = 8: 4096 atoms), next to a small structure; with the
    workspace of the bucket path (destination side through per-block buckets)
    and with the minimal workspace (global atomics)."""
    big = inputs.make_config5(B=1, m_lo=m, m_hi=m)
    small = inputs.random_batch(np.random.default_rng(30 + m), 2, 4, 30, 3.0, 7.0, cutoff=5.0)
    b = gu.concat([small, big], cutoff=5.0, k=16)
    g, (s, d, t, ln) = _edges(b)
    rng = np.random.default_rng(40 + m)
    gv = rng.normal(size=(len(s), 3)).astype(np.float32)
    glen = rng.normal(size=len(s)).astype(np.float32)
    L, X, P = gu.dev(b)
    run = graph.GeometryRunner(b.B, b.N, large=buckets)
    gf = torch.empty_like(X)
    gL = torch.empty_like(L)
    run.backward(L, X, P, g.src, g.dst, g.image, torch.from_numpy(gv).cuda(), torch.from_numpy(glen).cuda(), gf, gL)
    assert (run.workspace.numel() >= _lib.load().mg_geometry_backward_workspace_bytes(b.B, b.N, len(s))) == buckets
    rf, rL = oracle.edge_geometry_vjp64(b.lattices, b.frac, b.batch_ptr, s, d, t, gv, glen)
    _per_structure_check(b, gf.cpu().numpy(), gL.cpu().numpy(), rf, rL)


def test_backward_knn_edges():
    """KNN edges (k per source, source-major) with both upstream gradients."""
    b = inputs.make_config(4)
    g = gu.knn(b)
    s, d, t, ln = gu.np_graph(g)
    rng = np.random.default_rng(12)
    gv = rng.normal(size=(len(s), 3)).astype(np.float32)
    glen = rng.normal(size=len(s)).astype(np.float32)
    L, X, P = gu.dev(b)
    run = graph.GeometryRunner(b.B, b.N)
    gf = torch.empty_like(X)
    gL = torch.empty_like(L)
    run.backward(L, X, P, g.src, g.dst, g.image, torch.from_numpy(gv).cuda(), torch.from_numpy(glen).cuda(), gf, gL)
    rf, rL = oracle.edge_geometry_vjp64(b.lattices, b.frac, b.batch_ptr, s, d, t, gv, glen)
    _per_structure_check(b, gf.cpu().numpy(), gL.cpu().numpy(), rf, rL)


def test_backward_empty_structures_and_no_edges():
    """Structures without edges (isolated atoms far apart) get zero gradients;
    an empty edge list gives all-zero outputs."""
    b = gu.concat([gu.single(np.eye(3) * 20.0, [[0.1, 0.1, 0.1]]),
                   inputs.random_batch(np.random.default_rng(5), 2, 3, 10, 3.0, 6.0, cutoff=4.0),
                   gu.single(np.eye(3) * 30.0, [[0.5, 0.5, 0.5], [0.0, 0.0, 0.0]])], cutoff=4.0, k=4)
    g, (s, d, t, ln) = _edges(b)
    rng = np.random.default_rng(13)
    gv = rng.normal(size=(len(s), 3)).astype(np.float32)
    L, X, P = gu.dev(b)
    run = graph.GeometryRunner(b.B, b.N)
    gf = torch.full_like(X, 7.0)
    gL = torch.full_like(L, 7.0)
    run.backward(L, X, P, g.src, g.dst, g.image, torch.from_numpy(gv).cuda(), None, gf, gL)
    rf, rL = oracle.edge_geometry_vjp64(b.lattices, b.frac, b.batch_ptr, s, d, t, gv, None)
    gfn, gLn = gf.cpu().numpy(), gL.cpu().numpy()
    assert np.all(gfn[0] == 0) and np.all(gLn[0] == 0) and np.all(gfn[-2:] == 0) and np.all(gLn[-1] == 0)
    _per_structure_check(b, gfn, gLn, rf, rL)
    z = torch.zeros(0, dtype=torch.int32, device="cuda")
    run.backward(L, X, P, z, z, torch.zeros((0, 3), dtype=torch.int32, device="cuda"),
                 torch.zeros((0, 3), device="cuda"), None, gf, gL)
    assert float(gf.abs().max()) == 0.0 and float(gL.abs().max()) == 0.0


def test_backward_config4_sampled_finite_differences():
    """The 1024-structure differentiation workload: the GPU gradient of
    loss = sum_e w_e exp(-(l_e - 3)^2) (through the autograd function) against
    FP64 central differences (h = 1e-6) of sum_e (dloss/dl_e) l_e, on the fixed
    edge set, for 64 sampled atoms and 16 sampled lattices; error per entry at
    most 1e-4 of the largest oracle gradient entry of the structure."""
    b = inputs.make_config(4)
    g, (s, d, t, ln) = _edges(b)
    order = np.lexsort((t[:, 2], t[:, 1], t[:, 0], d, s))
    w = np.empty(len(s), np.float32)
    w[order] = inputs.loss_weights(len(s))
    L, X, P = gu.dev(b)
    L.requires_grad_(True)
    X.requires_grad_(True)
    vec, length = graph.edge_geometry(L, X, P, g.src, g.dst, g.image)
    loss = (torch.from_numpy(w).cuda() * torch.exp(-(length - 3.0) ** 2)).sum()
    loss.backward()
    gf, gL = X.grad.cpu().numpy(), L.grad.cpu().numpy()
    l64 = oracle.edge_geometry64(b.lattices, b.frac, b.batch_ptr, s, d, t)[1]
    gl64 = oracle.gaussian_loss_grad_len64(l64, w)
    gf64, gL64 = oracle.edge_geometry_vjp64(b.lattices, b.frac, b.batch_ptr, s, d, t, None, gl64)
    rng = np.random.default_rng(44)
    atoms = np.sort(rng.choice(b.N, 64, replace=False))
    structs = np.sort(rng.choice(b.B, 16, replace=False))
    # only the edges that touch a sampled atom or structure are needed by the differences
    s_of = np.searchsorted(b.batch_ptr, s, side="right") - 1
    keep = np.isin(s, atoms) | np.isin(d, atoms) | np.isin(s_of, structs)
    ff, fL = oracle.fd_vjp64(b.lattices, b.frac, b.batch_ptr, s[keep], d[keep], t[keep], None, gl64[keep],
                             h=1e-6, atoms=atoms.tolist(), structures=structs.tolist())
    worst = 0.0
    for a in atoms:
        q = int(np.searchsorted(b.batch_ptr, a, side="right")) - 1
        scale = max(np.abs(gf64[b.batch_ptr[q]:b.batch_ptr[q + 1]]).max(), 1e-300)
        worst = max(worst, np.abs(gf[a] - ff[a]).max() / scale)
    for q in structs:
        scale = max(np.abs(gL64[q]).max(), 1e-300)
        worst = max(worst, np.abs(gL[q] - fL[q]).max() / scale)
    print("worst relative error against finite differences", worst)
    assert worst <= 1e-4


def test_backward_supercell_shuffled_with_buckets():
    """A 1728-atom supercell whose edges are shuffled inside the structure,
    with the bucket path's workspace: the scatter pass finds the sources out
    of order, and the general kernel redoes the whole pass."""
    big = inputs.make_config5(B=1, m_lo=6, m_hi=6)
    small = inputs.random_batch(np.random.default_rng(36), 2, 4, 30, 3.0, 7.0, cutoff=5.0)
    b = gu.concat([small, big], cutoff=5.0, k=16)
    g, (s, d, t, ln) = _edges(b)
    rng = np.random.default_rng(46)
    blk = np.flatnonzero(s >= b.batch_ptr[2])
    perm = np.arange(len(s))
    perm[blk] = rng.permutation(blk)
    s, d, t = s[perm], d[perm], t[perm]
    glen = rng.normal(size=len(s)).astype(np.float32)
    L, X, P = gu.dev(b)
    run = graph.GeometryRunner(b.B, b.N, large=True)
    gf = torch.empty_like(X)
    gL = torch.empty_like(L)
    ti = lambda a: torch.from_numpy(np.ascontiguousarray(a.astype(np.int32))).cuda()
    run.backward(L, X, P, ti(s), ti(d), ti(t), None, torch.from_numpy(glen).cuda(), gf, gL)
    rf, rL = oracle.edge_geometry_vjp64(b.lattices, b.frac, b.batch_ptr, s, d, t, None, glen)
    _per_structure_check(b, gf.cpu().numpy(), gL.cpu().numpy(), rf, rL)
