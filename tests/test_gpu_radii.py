"""Per-atom cutoffs c_i (Definition def6: an edge uses its source's cutoff) on
the GPU against the FP64 oracle: closed form, random batches through both
image-sweep forms, and cell lists."""
import math

import numpy as np
import pytest
import torch

import compare
import gpu_util as gu
from paper_2307_05380_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def _radii_dev(r):
    return torch.from_numpy(np.ascontiguousarray(r, np.float32)).cuda()


def test_radii_cscl_closed_form():
    """CsCl arrangement, a = 1: c_A = 0.95 sees the 8 B at sqrt(3)/2; c_B = 1.05
    sees the 8 A and its 6 B images."""
    b = gu.single(np.eye(3), [[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]], cutoff=1.0)
    g = gu.cutoff(b, cutoff=_radii_dev([0.95, 1.05]))
    s, d, t, ln = gu.np_graph(g)
    assert np.bincount(s, minlength=2).tolist() == [8, 14]
    assert (d[s == 0] == 1).all()
    assert np.abs(ln[s == 0] - math.sqrt(3.0) / 2.0).max() <= 2e-6
    compare.cutoff_check(b, s, d, t, ln, radii=np.array([0.95, 1.05], np.float32))


@pytest.mark.parametrize("seed", [1, 2])
def test_radii_random_batch(seed):
    """Atom counts on both sides of 64 (both sweep forms); radii from a per-species
    table (8 species, 1.5-6 A), so sources of one structure differ."""
    rng = np.random.default_rng(100 + seed)
    b = inputs.random_batch(rng, 40, 1, 120, 3.0, 12.0, cutoff=5.0)
    table = rng.uniform(1.5, 6.0, size=8).astype(np.float32)
    radii = table[rng.integers(0, 8, size=b.N)]
    g = gu.cutoff(b, cutoff=_radii_dev(radii))
    assert g.report.flags == 0, g.report.flag_names()
    st = compare.cutoff_check(b, *gu.np_graph(g), radii=radii, processes=8)
    print(st)
    # equal radii give exactly the constant-cutoff graph (same kernels, same thresholds)
    ge = gu.cutoff(b, cutoff=_radii_dev(np.full(b.N, 5.0, np.float32)))
    gc = gu.cutoff(b, cutoff=5.0)
    for a, c in zip(gu.np_graph(ge), gu.np_graph(gc)):
        assert np.array_equal(a, c)


def test_radii_cell_lists():
    """Supercell through cell lists (forced and automatic) with per-species radii."""
    b = inputs.make_config5(B=1, m_lo=8, m_hi=8)
    rng = np.random.default_rng(7)
    table = rng.uniform(3.0, 5.0, size=8).astype(np.float32)
    radii = table[np.arange(b.N) % 8]
    g = gu.cutoff(b, cutoff=_radii_dev(radii))
    assert g.report.flags == 0, g.report.flag_names()
    s, d, t, ln = gu.np_graph(g)
    srcs = sorted(np.random.default_rng(8).choice(b.N, 48, replace=False).tolist())
    print(compare.cutoff_sources_check(b, 0, srcs, s, d, t, ln, radii=radii))
    gi = gu.cutoff(b, cutoff=_radii_dev(radii), opts=_lib.MG_OPT_CELL_LIST_OFF)
    a = compare._void(compare._rows(*gu.np_graph(gi)[:3]))
    c = compare._void(compare._rows(s, d, t))
    assert np.array_equal(np.sort(a), np.sort(c))


def test_radii_invalid_skips_structure():
    """A non-positive or NaN radius skips its structure (NONFINITE) and leaves the others intact."""
    rng = np.random.default_rng(9)
    b = inputs.random_batch(rng, 3, 4, 10, 4.0, 8.0, cutoff=5.0)
    radii = np.full(b.N, 5.0, np.float32)
    radii[b.batch_ptr[1]] = -1.0
    g = gu.cutoff(b, cutoff=_radii_dev(radii))
    assert g.report.flags & _lib.MG_FLAG_NONFINITE
    s, d, t, ln = gu.np_graph(g)
    assert not np.isin(s, np.arange(b.batch_ptr[1], b.batch_ptr[2])).any()
    compare.cutoff_check(b, s, d, t, ln, structures=[0, 2], radii=radii)
