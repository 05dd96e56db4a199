"""KNN multigraph on the GPU against the FP64 oracle (Sec. 1; Algorithms 1-2)."""
import itertools
import math

import numpy as np
import pytest

import compare
import gpu_util as gu
from paper_2307_05380_amd import inputs, _lib

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cfg", [1, 2])
def test_parity_full(cfg):
    b = inputs.make_config(cfg)
    g = gu.knn(b)
    assert g.report.flags & ~_lib.MG_FLAG_KNN_EXTENDED == 0, g.report.flag_names()
    st = compare.knn_check(b, b.k, *gu.np_graph(g), processes=8)
    print(st, g.report)


def test_parity_config3_sampled():
    b = inputs.make_config(3)
    g = gu.knn(b)
    assert g.report.flags & ~_lib.MG_FLAG_KNN_EXTENDED == 0, g.report.flag_names()
    rng = np.random.default_rng(3)
    n = b.counts()
    sample = sorted(set(rng.choice(b.B, 160, replace=False).tolist()) | set(np.argsort(-n)[:8].tolist())
                    | set(np.nonzero(n == 1)[0][:16].tolist()))
    st = compare.knn_check(b, b.k, *gu.np_graph(g), sources=sample, processes=8)
    print(st, g.report)


def test_tie_break_pins():
    """Exact ties are ordered by (dst, t lexicographic)."""
    g = gu.knn(gu.single(np.eye(3), np.zeros((1, 3))), k=8)
    want = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 1), (0, 1, 0), (1, 0, 0), (-1, -1, 0), (-1, 0, -1)]
    assert [tuple(int(q) for q in t) for t in g.image.cpu().numpy()] == want
    assert np.allclose(g.length.cpu().numpy(), [1] * 6 + [math.sqrt(2)] * 2, atol=1e-6)
    x = np.array([[0, 0, 0], [0.5, 0.5, 0.5]])
    g = gu.knn(gu.single(np.eye(3), x), k=10)
    d = g.dst.cpu().numpy().reshape(2, 10)
    t = [tuple(int(q) for q in r) for r in g.image.cpu().numpy()]
    assert (d[0, :8] == 1).all() and (d[1, :8] == 0).all()
    assert t[:8] == list(itertools.product((-1, 0), repeat=3))
    assert t[8:10] == [(-1, 0, 0), (0, -1, 0)]
    assert t[10:18] == list(itertools.product((0, 1), repeat=3))


def test_extended_search():
    """A tight cluster in a large cell: the density-based first radius misses,
    the extended search finds the images one cell away."""
    x = np.array([[0.5, 0.5, 0.5], [0.51, 0.5, 0.5], [0.5, 0.51, 0.5], [0.5, 0.5, 0.51]])
    b = gu.single(10.0 * np.eye(3), x, k=6)
    g = gu.knn(b)
    assert g.report.flags & _lib.MG_FLAG_KNN_EXTENDED
    compare.knn_check(b, 6, *gu.np_graph(g))


@pytest.mark.parametrize("k", [1, 5, 33, 64])
def test_k_range_random(k):
    rng = np.random.default_rng(20 + k)
    b = inputs.random_batch(rng, 24, 1, 90, 2.5, 12.0, cutoff=5.0, k=k)
    g = gu.knn(b)
    compare.knn_check(b, k, *gu.np_graph(g))


def test_single_atom_cells():
    rng = np.random.default_rng(9)
    b = inputs.random_batch(rng, 40, 1, 1, 2.5, 20.0, 30.0, 150.0, k=16)
    g = gu.knn(b)
    compare.knn_check(b, 16, *gu.np_graph(g))


@pytest.mark.parametrize("k", [33, 64])
def test_large_stacks_same_graph(k):
    """A wide first radius (lambda = 8) and no tighter first threshold push
    hundreds of keys per source: the ordered stack is compressed inside the
    sweep (sorting network) and more than 64 keys, two per lane, are ranked at
    the end. The graph must equal the oracle's and, bit for bit, the graph of
    the default search."""
    rng = np.random.default_rng(70 + k)
    b = inputs.random_batch(rng, 16, 20, 120, 4.0, 12.0, cutoff=5.0, k=k)
    ref = gu.np_graph(gu.knn(b))
    saved = _lib.get_tuning()
    try:
        _lib.set_tuning(**dict(saved, knn_lambda_x4=32, knn_tau_x8=64))
        g = gu.knn(b)
    finally:
        _lib.set_tuning(**saved)
    assert g.report.flags & ~_lib.MG_FLAG_KNN_EXTENDED == 0, g.report.flag_names()
    got = gu.np_graph(g)
    for x, y in zip(ref, got):
        assert np.array_equal(x, y)
    compare.knn_check(b, k, *got)
