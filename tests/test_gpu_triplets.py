"""Triplets Gamma_2 on the GPU against the oracle: pair lists exactly, angles
to FP32 rounding; cutoff graphs (row_ptr from the builder) and KNN graphs."""
import numpy as np
import pytest
import torch

import gpu_util as gu
import oracle
from paper_2307_05380_amd import graph, inputs

pytestmark = pytest.mark.gpu


def _check(row_ptr, E, vec_dev, tr, cos_tol=2e-6):
    ptr = row_ptr.cpu().numpy()
    o1, o2 = oracle.triplets64(ptr)
    assert tr.report.num_edges == len(o1) and tr.report.flags == 0
    assert np.array_equal(tr.e1.cpu().numpy(), o1) and np.array_equal(tr.e2.cpu().numpy(), o2)
    d = np.diff(ptr)
    assert np.array_equal(np.diff(tr.trip_ptr.cpu().numpy()), d * (d - 1))
    if vec_dev is not None:
        oc = oracle.triplet_cos64(vec_dev.cpu().numpy(), o1, o2)
        assert np.abs(tr.cos_theta.cpu().numpy() - oc).max(initial=0.0) <= cos_tol


def test_triplets_cutoff_graph():
    rng = np.random.default_rng(50)
    b = inputs.random_batch(rng, 30, 1, 40, 3.0, 9.0, cutoff=4.0)
    g = gu.cutoff(b)
    L, X, P = gu.dev(b)
    vec, _ = graph.GeometryRunner(b.B, b.N).forward(L, X, P, g.src, g.dst, g.image,
                                                     torch.empty((g.num_edges, 3), device="cuda"),
                                                     torch.empty(g.num_edges, device="cuda"))
    tr = graph.triplets(g.row_ptr, g.num_edges, vec)
    _check(g.row_ptr, g.num_edges, vec, tr)


def test_triplets_knn_graph_and_capacity_retry():
    b = inputs.make_config(4)
    g = gu.knn(b)
    k = b.k
    row_ptr = torch.arange(0, b.N * k + 1, k, dtype=torch.int64, device="cuda")
    tr = graph.triplets(row_ptr, b.N * k, None, capacity=1000)     # too small: reruns
    _check(row_ptr, b.N * k, None, tr)
    assert tr.cos_theta is None


def test_triplets_degenerate_and_invalid():
    # degrees 0, 1, 2, 5; then a decreasing row_ptr flags RANGE and yields nothing for that source
    row_ptr = torch.tensor([0, 0, 1, 3, 8], dtype=torch.int64, device="cuda")
    tr = graph.triplets(row_ptr, 8)
    _check(row_ptr, 8, None, tr)
    bad = torch.tensor([0, 4, 2, 6], dtype=torch.int64, device="cuda")
    tr = graph.triplets(bad, 6)
    assert tr.report.flags & 16                     # MG_FLAG_RANGE
    assert tr.report.num_edges == 2 * 4 * 3         # sources 0 and 2 are valid ranges
    empty = torch.zeros(1, dtype=torch.int64, device="cuda")
    tr = graph.triplets(empty, 0)
    assert tr.report.num_edges == 0 and tr.e1.numel() == 0
