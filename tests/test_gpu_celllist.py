"""Cell lists for large structures on the GPU (supercells of the 64-supercell
update workload, forced cell lists on large cells, wrapped coordinates),
checked against the FP64 oracle on sampled sources."""
import numpy as np
import pytest

import compare
import gpu_util as gu
from paper_2307_05380_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def _sample(n, count, seed):
    rng = np.random.default_rng(seed)
    return sorted(rng.choice(n, min(count, n), replace=False).tolist())


@pytest.fixture(scope="module")
def supercells():
    # two supercells (8x8x8 and 9x9x9 tilings of an 8-atom cell), 4096 and 5832 atoms
    return inputs.make_config5(B=2, m_lo=8, m_hi=9)


class _span:
    """Cell-list stencil half-width for the calls inside the block (1: 27 bins, 2: 125 bins)."""

    def __init__(self, span):
        self.span = span

    def __enter__(self):
        self.saved = _lib.get_tuning()
        _lib.set_tuning(**dict(self.saved, cutoff_cl_span=self.span, knn_cl_span=self.span))

    def __exit__(self, *a):
        _lib.set_tuning(**self.saved)


@pytest.mark.parametrize("span", [1, 2])
def test_supercell_cutoff_cell_lists(supercells, span):
    b = supercells
    with _span(span):
        g = gu.cutoff(b)
    assert g.report.flags == 0, g.report.flag_names()
    s, d, t, ln = gu.np_graph(g)
    for q in range(b.B):
        n = int(b.batch_ptr[q + 1] - b.batch_ptr[q])
        st = compare.cutoff_sources_check(b, q, _sample(n, 48, q), s, d, t, ln)
        print(q, st)
    rp = g.row_ptr.cpu().numpy()
    assert np.array_equal(np.repeat(np.arange(b.N), np.diff(rp)), s)


@pytest.mark.parametrize("k", [32, 64])
def test_supercell_knn_large_stacks_same_graph(supercells, k):
    """A wide search radius (lambda = 8: stencils beyond what the tile stages,
    candidates read from the slot arrays) and no tighter first threshold push
    hundreds of staged keys per source: the cell-list stack keeps only the keys
    near its k-th inside the sweep, and more than 64 keys are ranked two per
    lane. The graph must equal the default search's bit for bit and the
    oracle's on sampled sources."""
    b = supercells
    ref = gu.np_graph(gu.knn(b, k=k))
    saved = _lib.get_tuning()
    try:
        _lib.set_tuning(**dict(saved, knn_lambda_x4=32, knn_tau_x8=64))
        g = gu.knn(b, k=k)
    finally:
        _lib.set_tuning(**saved)
    assert g.report.flags & ~_lib.MG_FLAG_KNN_EXTENDED == 0, g.report.flag_names()
    got = gu.np_graph(g)
    for x, y in zip(ref, got):
        assert np.array_equal(x, y)
    s, d, t, ln = got
    for q in range(b.B):
        n = int(b.batch_ptr[q + 1] - b.batch_ptr[q])
        compare.knn_sources_check(b, q, k, _sample(n, 16, 30 + q), s, d, t, ln)


@pytest.mark.parametrize("span", [1, 2])
def test_supercell_knn_cell_lists(supercells, span):
    b = supercells
    with _span(span):
        g = gu.knn(b, k=32)
    assert g.report.flags & ~_lib.MG_FLAG_KNN_EXTENDED == 0, g.report.flag_names()
    s, d, t, ln = gu.np_graph(g)
    for q in range(b.B):
        n = int(b.batch_ptr[q + 1] - b.batch_ptr[q])
        compare.knn_sources_check(b, q, 32, _sample(n, 48, 10 + q), s, d, t, ln)
    print(g.report)


def test_stencil_spans_same_graph(supercells):
    """27-bin and 125-bin stencils build the same cutoff edge set (lengths
    within the length tolerance: the staged positions are rounded relative to
    bins of another size) and bit-identical KNN graphs."""
    b = supercells
    out = {}
    for span in (1, 2):
        with _span(span):
            out[span] = (gu.np_graph(gu.cutoff(b)), gu.np_graph(gu.knn(b, k=32)))
    (c1, k1), (c2, k2) = out[1], out[2]
    for x, y in zip(k1, k2):
        assert np.array_equal(x, y)

    def keyed(e):
        s, d, t, ln = e
        return dict(zip(zip(s.tolist(), d.tolist(), map(tuple, t.tolist())), ln.tolist()))
    a, c = keyed(c1), keyed(c2)
    assert a.keys() == c.keys()
    assert max(abs(a[q] - c[q]) for q in a) <= compare.LEN_TOL


def _large_cells(seed, B=6):
    rng = np.random.default_rng(seed)
    return inputs.random_batch(rng, B, 40, 220, 15.0, 26.0, 60.0, 120.0, cutoff=5.0, k=12)


@pytest.mark.parametrize("span", [1, 2])
def test_forced_cell_lists_match_image_sweep(span):
    """The same batch through cell lists (forced) and through the image sweep:
    both agree with the oracle and give the same edge set, the band of the
    cutoff included (the cell-list sweep decides candidates near the threshold
    in the image sweep's arithmetic); the lengths of common edges agree to twice
    the length tolerance, and the KNN graphs bit for bit."""
    b = _large_cells(3)
    with _span(span):
        gc = gu.cutoff(b, opts=_lib.MG_OPT_CELL_LIST_FORCE)
        kc_ = gu.knn(b, opts=_lib.MG_OPT_CELL_LIST_FORCE)
    gi = gu.cutoff(b, opts=_lib.MG_OPT_CELL_LIST_OFF)
    ec, ei = gu.np_graph(gc), gu.np_graph(gi)
    compare.cutoff_check(b, *ec)
    compare.cutoff_check(b, *ei)

    def keyed(e):
        s, d, t, ln = e
        return {(int(a), int(c), int(x), int(y), int(z)): float(l) for a, c, (x, y, z), l in zip(s, d, t, ln)}
    kc, ki = keyed(ec), keyed(ei)
    assert set(kc) == set(ki), f"paths differ: {sorted(set(kc) ^ set(ki))[:3]}"
    assert max(abs(kc[k] - ki[k]) for k in kc) <= 2 * compare.LEN_TOL
    ki_ = gu.knn(b, opts=_lib.MG_OPT_CELL_LIST_OFF)
    compare.knn_check(b, b.k, *gu.np_graph(kc_))
    for x, y in zip(gu.np_graph(kc_), gu.np_graph(ki_)):
        assert np.array_equal(x, y)


def test_cell_lists_wrapped_coordinates():
    b = _large_cells(4)
    rng = np.random.default_rng(0)
    shift = rng.integers(-2, 3, size=b.frac.shape).astype(np.float32)
    b.frac[:] = b.frac + shift
    g = gu.cutoff(b, opts=_lib.MG_OPT_CELL_LIST_FORCE)
    compare.cutoff_check(b, *gu.np_graph(g))
    k = gu.knn(b, opts=_lib.MG_OPT_CELL_LIST_FORCE)
    compare.knn_check(b, b.k, *gu.np_graph(k))


def test_cell_lists_far_coordinates():
    """Coordinates hundreds of cells away from [0, 1) (beyond what the cell
    lists' packed cell index holds): the structure goes through the image sweep
    and its edges still match the oracle, with t relative to the coordinates
    as given. Def. def6 is invariant under x_a -> x_a + s_a (s_a integer):
    edge (i, j, t) of the shifted coordinates is edge (i, j, t + s_j - s_i) of
    the unshifted ones, so the oracle runs on the unshifted batch (its union
    of per-pair image ranges would span the whole 1200-cell shift) and the GPU
    edges are mapped back. Both batches hold the same FP32 values up to the
    exact integer shift."""
    b = _large_cells(5, B=3)
    rng = np.random.default_rng(1)
    shift = rng.choice([-600.0, 0.0, 600.0], size=b.frac.shape).astype(np.float32)
    far = inputs.Batch(b.lattices.copy(), (b.frac + shift).astype(np.float32), b.batch_ptr.copy(),
                       b.cutoff, b.k, "far")
    near = inputs.Batch(b.lattices, (far.frac - shift).astype(np.float32), b.batch_ptr, b.cutoff, b.k, "near")
    assert np.array_equal(far.frac.astype(np.float64) - shift, near.frac.astype(np.float64))   # exact
    s_int = shift.astype(np.int64)

    def back(g):
        s, d, t, ln = gu.np_graph(g)
        return s, d, t + s_int[d] - s_int[s], ln

    g = gu.cutoff(far, opts=_lib.MG_OPT_CELL_LIST_FORCE)
    assert g.report.flags == 0, g.report.flag_names()
    compare.cutoff_check(near, *back(g))
    k = gu.knn(far, opts=_lib.MG_OPT_CELL_LIST_FORCE)
    assert k.report.flags & ~_lib.MG_FLAG_KNN_EXTENDED == 0, k.report.flag_names()
    compare.knn_check(near, near.k, *back(k))


def test_cell_list_knn_extended():
    """Clustered atoms: the k-th neighbour lies beyond the stencil, the source
    falls back to the extended search."""
    rng = np.random.default_rng(7)
    L = 30.0 * np.eye(3, dtype=np.float32)
    x = np.concatenate([0.5 + 0.004 * rng.standard_normal((6, 3)), rng.random((200, 3))]).astype(np.float32)
    b = gu.single(L, x, cutoff=5.0, k=12)
    g = gu.knn(b, opts=_lib.MG_OPT_CELL_LIST_FORCE)
    compare.knn_check(b, 12, *gu.np_graph(g))
