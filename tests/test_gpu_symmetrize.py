"""Symmetric closure on the GPU against the oracle: KNN graphs (exact edge
lists in the documented order, lengths copied bit for bit), symmetric cutoff
graphs unchanged, malformed row pointers and capacity reruns."""
import numpy as np
import pytest
import torch

import gpu_util as gu
import oracle
from paper_2307_05380_amd import _lib, graph, inputs

pytestmark = pytest.mark.gpu


def _check(row_ptr, dst, image, length, g):
    op, os_, od, oi, ol = oracle.symmetrize64(row_ptr.cpu().numpy(), dst.cpu().numpy(), image.cpu().numpy(),
                                              None if length is None else length.cpu().numpy())
    assert g.report.num_edges == len(os_)
    assert np.array_equal(g.row_ptr.cpu().numpy(), op)
    assert np.array_equal(g.src.cpu().numpy(), os_)
    assert np.array_equal(g.dst.cpu().numpy(), od)
    assert np.array_equal(g.image.cpu().numpy(), oi)
    if length is not None:
        assert np.array_equal(g.length.cpu().numpy(), ol)


@pytest.mark.parametrize("which", ["config4", "small_cells"])
def test_symmetrize_knn(which):
    if which == "config4":
        b = inputs.make_config(4)
    else:   # small cells: many self-image edges (i, i, t)
        b = inputs.random_batch(np.random.default_rng(60), 64, 1, 6, 2.5, 5.0, cutoff=5.0, k=12)
    g = gu.knn(b)
    k = b.k
    row_ptr = torch.arange(0, b.N * k + 1, k, dtype=torch.int64, device="cuda")
    s = graph.symmetrize(row_ptr, g.dst, g.image, g.length)
    assert s.report.flags == 0
    _check(row_ptr, g.dst, g.image, g.length, s)
    added = s.report.num_edges - b.N * k
    print("added reverse edges", added, "of", b.N * k)
    assert added > 0


def test_symmetrize_cutoff_graph_unchanged():
    b = inputs.make_config(4)
    g = gu.cutoff(b)
    s = graph.symmetrize(g.row_ptr, g.dst, g.image, g.length)
    assert s.report.num_edges == g.num_edges
    for a, c in ((s.src, g.src), (s.dst, g.dst), (s.image, g.image), (s.length, g.length), (s.row_ptr, g.row_ptr)):
        assert torch.equal(a, c)


def test_symmetrize_capacity_and_malformed():
    b = inputs.random_batch(np.random.default_rng(61), 8, 2, 10, 3.0, 6.0, cutoff=5.0, k=4)
    g = gu.knn(b)
    row_ptr = torch.arange(0, b.N * 4 + 1, 4, dtype=torch.int64, device="cuda")
    s = graph.symmetrize(row_ptr, g.dst, g.image, None, capacity=3)      # too small: reruns
    _check(row_ptr, g.dst, g.image, None, s)
    assert s.length is None
    bad = row_ptr.clone()
    bad[2] = 10 ** 9                                                      # past E: clamped
    s = graph.symmetrize(bad, g.dst, g.image, None)
    assert s.report.flags & _lib.MG_FLAG_RANGE
    z = torch.zeros(1, dtype=torch.int64, device="cuda")
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    s = graph.symmetrize(z, e, torch.zeros((0, 3), dtype=torch.int32, device="cuda"))
    assert s.report.num_edges == 0
