"""Seeded synthetic inputs: determinism, shapes, dtypes and sampling rules (CPU)."""
import math

import numpy as np
import pytest

from paper_2307_05380_amd import inputs


@pytest.mark.parametrize("cfg", [1, 2, 3, 4])
def test_deterministic_and_layout(cfg):
    a = inputs.make_config(cfg)
    b = inputs.make_config(cfg)
    assert np.array_equal(a.lattices, b.lattices) and np.array_equal(a.frac, b.frac)
    assert np.array_equal(a.batch_ptr, b.batch_ptr)
    assert a.lattices.dtype == np.float32 and a.lattices.shape == (a.B, 3, 3)
    assert a.frac.dtype == np.float32 and a.frac.shape == (a.N, 3)
    assert a.batch_ptr.dtype == np.int64 and a.batch_ptr[0] == 0 and a.batch_ptr[-1] == a.N
    assert (np.diff(a.batch_ptr) >= 1).all()
    assert (a.frac >= 0).all() and (a.frac < 1).all()
    assert (np.linalg.det(a.lattices.astype(np.float64)) > 0).all()


def test_config_rules():
    c1 = inputs.make_config(1)
    assert c1.B == 1 and c1.N == 16 and c1.cutoff == 6.0 and c1.k == 12
    assert np.abs(c1.lattices[0] / 5.0 - np.eye(3)).max() <= 0.1 + 1e-6
    c2 = inputs.make_config(2)
    n = c2.counts()
    assert c2.B == 256 and n.min() >= 4 and n.max() <= 64
    ln = np.linalg.norm(c2.lattices.astype(np.float64), axis=2)
    assert ln.min() >= 3.0 - 1e-5 and ln.max() <= 15.0 + 1e-5
    c3 = inputs.make_config(3)
    n = c3.counts()
    assert c3.B == 4096 and n.min() >= 1 and n.max() <= 128 and c3.cutoff == 8.0 and c3.k == 16
    # log-uniform atom counts: about ln 2 / ln 129 of the structures have one atom
    assert abs((n == 1).mean() - math.log(2) / math.log(129)) < 0.03
    L = c3.lattices.astype(np.float64)
    ln = np.linalg.norm(L, axis=2)
    vf = np.abs(np.linalg.det(L)) / ln.prod(axis=1)
    assert vf.min() >= 0.05 - 1e-4
    assert ln.min() >= 2.5 - 1e-5 and ln.max() <= 20.0 + 1e-5


def test_config5_small():
    b = inputs.make_config5(B=2, m_lo=2, m_hi=3)
    n = b.counts()
    assert set(n.tolist()) <= {8 * 8, 8 * 27}
    d = inputs.config5_step_delta(b, 3)
    assert d.shape == (b.N, 3) and d.dtype == np.float32
    assert np.array_equal(d, inputs.config5_step_delta(b, 3))
    assert not np.array_equal(d, inputs.config5_step_delta(b, 4))


def test_subset_and_weights():
    b = inputs.make_config(2)
    s = b.subset([5, 2])
    assert s.B == 2 and np.array_equal(s.lattices[0], b.lattices[5])
    assert np.array_equal(s.frac[:s.batch_ptr[1]], b.frac[b.batch_ptr[5]:b.batch_ptr[6]])
    w = inputs.loss_weights(100)
    assert w.dtype == np.float32 and np.array_equal(w, inputs.loss_weights(100))


def test_cell_from_parameters():
    L = inputs.cell_from_parameters(3.0, 4.0, 5.0, *np.deg2rad([70.0, 80.0, 100.0]))
    assert np.allclose(np.linalg.norm(L, axis=1), [3, 4, 5])
    cosg = L[0] @ L[1] / 12.0
    cosb = L[0] @ L[2] / 15.0
    cosa = L[1] @ L[2] / 20.0
    assert np.allclose([cosa, cosb, cosg], np.cos(np.deg2rad([70.0, 80.0, 100.0])))
