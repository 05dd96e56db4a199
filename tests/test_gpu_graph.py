"""The whole hot path captured once in a HIP graph and replayed: every replay,
with new coordinates written between replays by eager work, must reproduce an
eager run of the same step (edge lists exactly, gradients to rounding)."""
import numpy as np
import pytest
import torch

import gpu_util as gu
from paper_2307_05380_amd import _lib, graph, inputs

pytestmark = pytest.mark.gpu


def _outputs(cb, kb, length, gf, gL):
    rep = cb.report()
    E = rep.num_edges
    return rep, [t.clone() for t in (cb.src[:E], cb.dst[:E], cb.image[:E], length[:E], kb.src, kb.dst, kb.image,
                                     kb.length, gf, gL)]


@pytest.mark.parametrize("opts", [_lib.MG_OPT_CELL_LIST_OFF, _lib.MG_OPT_CELL_LIST_FORCE])
def test_graph_replay_matches_eager(opts):
    rng = np.random.default_rng(21)
    b = inputs.random_batch(rng, 48, 1, 40, 3.0, 10.0, cutoff=5.0, k=12)
    L, X, P = gu.dev(b)
    X0 = X.clone()
    g = gu.cutoff(b)
    cap = 2 * g.num_edges + 1024
    cb = graph.CutoffBuilder(b.B, b.N, cap, 4 * g.report.images_needed + 4096, X.device)
    kb = graph.KnnBuilder(b.B, b.N, b.k, 64 * b.B + 4096, X.device)
    geo = graph.GeometryRunner(b.B, b.N, X.device)
    vec = torch.empty((cap, 3), device=X.device)
    length = torch.empty(cap, device=X.device)
    gf = torch.empty_like(X)
    gL = torch.empty_like(L)
    glen = torch.from_numpy(rng.normal(size=cap).astype(np.float32)).cuda()
    ne = cb.rep[:1]

    def step():
        cb.run(L, X, P, b.cutoff, opts)
        kb.run(L, X, P, opts)
        geo.forward(L, X, P, cb.src, cb.dst, cb.image, vec, length, num_edges=ne)
        geo.backward(L, X, P, cb.src, cb.dst, cb.image, None, glen, gf, gL, num_edges=ne)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    cg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cg):
        step()
    torch.cuda.synchronize()
    sizes = set()
    for r in range(4):
        # eager work between replays: move the atoms
        d = torch.from_numpy(rng.normal(0.0, 0.01, size=tuple(X.shape)).astype(np.float32)).cuda()
        X.copy_(X0 + r * d)
        torch.cuda.synchronize()
        cg.replay()
        torch.cuda.synchronize()
        rep_g, out_g = _outputs(cb, kb, length, gf, gL)
        step()
        torch.cuda.synchronize()
        rep_e, out_e = _outputs(cb, kb, length, gf, gL)
        assert rep_g.flags & ~_lib.MG_FLAG_KNN_EXTENDED == 0, rep_g.flag_names()
        assert rep_g.num_edges == rep_e.num_edges and rep_g.candidates == rep_e.candidates
        sizes.add(rep_g.num_edges)
        for a, e in zip(out_g[:8], out_e[:8]):
            assert torch.equal(a, e)
        for a, e in zip(out_g[8:], out_e[8:]):
            assert float((a - e).abs().max()) <= 1e-5 * max(float(e.abs().max()), 1e-30)
    assert len(sizes) >= 2   # the moves changed the edge count, and the replay followed


def test_two_stream_step_with_edge_vectors():
    """The benchmarked form of the step: the cutoff build writes the edge vectors,
    the KNN build runs on a second stream that forks from and joins the main
    one, the whole step captured once and replayed with moved atoms. Every
    replay must equal a one-stream eager run of the same calls."""
    rng = np.random.default_rng(29)
    b = inputs.random_batch(rng, 48, 1, 40, 3.0, 10.0, cutoff=5.0, k=12)
    L, X, P = gu.dev(b)
    X0 = X.clone()
    g = gu.cutoff(b)
    cap = 2 * g.num_edges + 1024
    opts = _lib.MG_OPT_CELL_LIST_OFF
    cb = graph.CutoffBuilder(b.B, b.N, cap, 4 * g.report.images_needed + 4096, X.device, vec=True)
    kb = graph.KnnBuilder(b.B, b.N, b.k, 64 * b.B + 4096, X.device)
    geo = graph.GeometryRunner(b.B, b.N, X.device)
    gf = torch.empty_like(X)
    gL = torch.empty_like(L)
    glen = torch.from_numpy(rng.normal(size=cap).astype(np.float32)).cuda()
    ne = cb.rep[:1]
    ks = torch.cuda.Stream()

    def step_two():
        main = torch.cuda.current_stream()
        ks.wait_stream(main)
        with torch.cuda.stream(ks):
            kb.run(L, X, P, opts)
        cb.run(L, X, P, b.cutoff, opts)
        geo.backward(L, X, P, cb.src, cb.dst, cb.image, None, glen, gf, gL, num_edges=ne)
        main.wait_stream(ks)

    def step_one():
        cb.run(L, X, P, b.cutoff, opts)
        kb.run(L, X, P, opts)
        geo.backward(L, X, P, cb.src, cb.dst, cb.image, None, glen, gf, gL, num_edges=ne)

    def outputs():
        rep = cb.report()
        E = rep.num_edges
        return rep, [t.clone() for t in (cb.src[:E], cb.dst[:E], cb.image[:E], cb.length[:E], cb.vec[:E], kb.src,
                                         kb.dst, kb.image, kb.length, gf, gL)]

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step_two()
    torch.cuda.current_stream().wait_stream(side)
    cg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cg):
        step_two()
    torch.cuda.synchronize()
    for r in range(3):
        d = torch.from_numpy(rng.normal(0.0, 0.01, size=tuple(X.shape)).astype(np.float32)).cuda()
        X.copy_(X0 + r * d)
        torch.cuda.synchronize()
        cg.replay()
        torch.cuda.synchronize()
        rep_g, out_g = outputs()
        step_one()
        torch.cuda.synchronize()
        rep_e, out_e = outputs()
        assert rep_g.flags & ~_lib.MG_FLAG_KNN_EXTENDED == 0, rep_g.flag_names()
        assert rep_g.num_edges == rep_e.num_edges
        for a, e in zip(out_g[:9], out_e[:9]):
            assert torch.equal(a, e)
        for a, e in zip(out_g[9:], out_e[9:]):
            assert float((a - e).abs().max()) <= 1e-5 * max(float(e.abs().max()), 1e-30)
