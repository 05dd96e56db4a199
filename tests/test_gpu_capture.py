"""Sizing before capture and the overflow protocol of a captured step: the
image-slot query and the count-only cutoff call give the sizes a full call
reports; a captured step whose builders are too small (or become too small
when the atoms move) is grown, captured again and replayed, and then equals
an eager run."""
import numpy as np
import pytest
import torch

import gpu_util as gu
from paper_2307_05380_amd import _lib, graph, inputs

pytestmark = pytest.mark.gpu


def _batch():
    return inputs.make_config2(B=64)


def test_images_needed_and_sizes_match_full_calls():
    b = _batch()
    L, X, P = gu.dev(b)
    g = graph.cutoff_graph(L, X, P, b.cutoff, opts=_lib.MG_OPT_CELL_LIST_OFF)
    kn = graph.knn_graph(L, X, P, b.k, opts=_lib.MG_OPT_CELL_LIST_OFF)
    rc = graph.images_needed(L, X, P, b.cutoff, opts=_lib.MG_OPT_CELL_LIST_OFF)
    rk = graph.images_needed(L, X, P, k=b.k, opts=_lib.MG_OPT_CELL_LIST_OFF)
    assert rc.images_needed == g.report.images_needed and rc.flags == 0 and rc.num_edges == 0
    assert rk.images_needed == kn.report.images_needed and rk.flags == 0
    E, icap = graph.cutoff_sizes(L, X, P, b.cutoff, opts=_lib.MG_OPT_CELL_LIST_OFF)
    assert E == g.num_edges and icap == g.report.images_needed
    # per-atom cutoffs
    radii = torch.full((b.N,), 5.0, dtype=torch.float32, device="cuda")
    rr = graph.images_needed(L, X, P, radii, opts=_lib.MG_OPT_CELL_LIST_OFF)
    gr = graph.cutoff_graph(L, X, P, radii, opts=_lib.MG_OPT_CELL_LIST_OFF)
    assert rr.images_needed == gr.report.images_needed


def _sorted_edges(src, dst, img):
    a = np.concatenate([src[:, None], dst[:, None], img], 1).astype(np.int64)
    return a[np.lexsort(a.T[::-1])]


def test_captured_step_recaptures_on_overflow():
    print("captured step: 64 structures, tiny capacities, then compressed lattices", flush=True)
    b = _batch()
    L, X, P = gu.dev(b)
    opts = _lib.MG_OPT_CELL_LIST_OFF
    cb = graph.CutoffBuilder(b.B, b.N, 1000, 64, "cuda", vec=True)      # far too small
    kb = graph.KnnBuilder(b.B, b.N, b.k, 64, "cuda")
    Lrun = L.clone()

    def step():
        cb.run(Lrun, X, P, b.cutoff, opts)
        kb.run(Lrun, X, P, opts)

    cs = graph.CapturedStep(step, [cb, kb])
    assert cs.replay(check=True)          # grown and captured again
    assert cs.recaptures >= 1
    for scale in (1.0, 0.93):             # a denser batch needs more edges and images: another recapture
        Lrun.copy_(L * scale)
        cs.replay(check=True)
        rc, rk = cb.report(), kb.report()
        assert not cb.overflowed(rc) and not kb.overflowed(rk)
        ge = graph.cutoff_graph(Lrun, X, P, b.cutoff, opts=opts)
        ke = graph.knn_graph(Lrun, X, P, b.k, opts=opts)
        got = cb.graph(rc)
        assert got.num_edges == ge.num_edges
        np.testing.assert_array_equal(got.row_ptr.cpu().numpy(), ge.row_ptr.cpu().numpy())
        np.testing.assert_array_equal(_sorted_edges(*gu.np_graph(got)[:3]), _sorted_edges(*gu.np_graph(ge)[:3]))
        for a, e in zip((kb.dst, kb.image, kb.length), (ke.dst, ke.image, ke.length)):
            assert torch.equal(a, e)
    assert cs.recaptures >= 2
