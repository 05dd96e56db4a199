"""KNN with ties kept (Algorithm 2's d <= d_k) on the GPU: whole coordination
shells of ideal crystals (exact ties in FP32), against the oracle, and equal to
the exact-k graph when there are no ties."""
import math

import numpy as np
import pytest
import torch

import gpu_util as gu
import oracle
from paper_2307_05380_amd import _lib, graph, inputs

pytestmark = pytest.mark.gpu


def _ties(b, k, **kw):
    L, X, P = gu.dev(b)
    g = graph.knn_graph_ties(L, X, P, k, **kw)
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("name,frac,k,want", [
    ("sc", [[0.0, 0.0, 0.0]], 4, 6),
    ("sc", [[0.0, 0.0, 0.0]], 7, 18),
    ("bcc", [[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]], 3, 8),
    ("fcc", [[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]], 13, 18),
])
def test_ties_shells(name, frac, k, want):
    b = gu.single(3.0 * np.eye(3), frac, k=k)
    g = _ties(b, k)
    assert g.report.flags & ~_lib.MG_FLAG_KNN_EXTENDED == 0, g.report.flag_names()
    rp = g.row_ptr.cpu().numpy()
    assert np.diff(rp).tolist() == [want] * len(frac)
    s, d, t, ln = gu.np_graph(g)
    os_, od, ot, ol, optr = oracle.knn_ties_structure64(b.lattices[0], b.frac, k)
    assert np.array_equal(optr, rp)
    assert np.array_equal(d, od) and np.array_equal(t, ot)
    assert np.abs(ln - ol).max() <= 2e-5


def test_ties_generic_equals_knn():
    rng = np.random.default_rng(70)
    b = inputs.random_batch(rng, 40, 1, 60, 3.0, 10.0, cutoff=5.0, k=12)
    g = _ties(b, 12)
    kg = gu.knn(b)
    assert g.report.num_edges == b.N * 12
    assert torch.equal(g.row_ptr, torch.arange(0, b.N * 12 + 1, 12, device="cuda"))
    for a, c in zip(gu.np_graph(g), gu.np_graph(kg)):
        assert np.array_equal(a, c)


def test_ties_capacity_and_truncation():
    # sc with k = 1: 6 ties; a capacity of 2 forces the rerun
    b = gu.single(3.0 * np.eye(3), [[0.0, 0.0, 0.0]], k=1)
    g = _ties(b, 1, capacity=2)
    assert g.report.num_edges == 6 and np.diff(g.row_ptr.cpu().numpy()).tolist() == [6]
    # sc with k = 60: shells of 6, 12, 8, 6, 24, 24 neighbours (cumulative 56, 80), so the
    # 60th lies in the sqrt(6) shell and its ties run to 80 > 64 keys -> truncated, flagged
    g = _ties(b, 60)
    assert g.report.flags & _lib.MG_FLAG_TIES
    assert g.report.num_edges == 64
