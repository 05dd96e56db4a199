"""Autotuner on the GPU: every candidate yields the same graph, the best
parameters round-trip through the cache and leave the library's results
unchanged."""
import numpy as np
import pytest
import torch

import gpu_util as gu
from paper_2307_05380_amd import _lib, inputs, tune

pytestmark = pytest.mark.gpu


def test_tune_and_cache(tmp_path, monkeypatch):
    monkeypatch.setenv("MG_TUNE_CACHE", str(tmp_path / "tune.json"))
    rng = np.random.default_rng(33)
    # sizes on both sides of 64 atoms: both sweep forms and all slot widths run
    b = inputs.random_batch(rng, 24, 1, 150, 4.0, 12.0, cutoff=6.0, k=16)
    L, X, P = gu.dev(b)
    base = _lib.get_tuning()
    try:
        ref_c = gu.cutoff(b)
        ref_k = gu.knn(b)
        best = tune.autotune(L, X, P, b.cutoff, b.k, reps=2)
        assert set(best["cutoff"]) == {"cutoff_wgs_per_cu", "cutoff_slots", "cutoff_img_group"}
        assert set(best["knn"]) == {"knn_wgs_per_cu", "knn_lambda_x4", "knn_tau_x8"}
        cur = _lib.get_tuning()
        for key, v in {**best["cutoff"], **best["knn"]}.items():
            assert cur[key] == v
        # cached: a second call loads instead of tuning
        again = tune.autotune(L, X, P, b.cutoff, b.k, reps=2)
        assert again["cutoff"] == best["cutoff"] and again["knn"] == best["knn"]
        # the tuned library builds the same graphs
        g = gu.cutoff(b)
        k = gu.knn(b)
        assert torch.equal(g.row_ptr, ref_c.row_ptr)
        for a, r in zip(gu.np_graph(k), gu.np_graph(ref_k)):
            assert np.array_equal(a, r)
        ga = sorted(zip(*[x.tolist() if x.ndim == 1 else [tuple(r) for r in x.tolist()] for x in gu.np_graph(g)]))
        gr = sorted(zip(*[x.tolist() if x.ndim == 1 else [tuple(r) for r in x.tolist()] for x in gu.np_graph(ref_c)]))
        assert ga == gr
    finally:
        _lib.set_tuning(**base)


def test_tune_cell_list_spans():
    """With cell-list structures in the batch the stencil half-widths join the
    search; every candidate (27- or 125-bin stencils) gives the same graph."""
    b = inputs.make_config5(B=2, m_lo=8, m_hi=8)
    L, X, P = gu.dev(b)
    base = _lib.get_tuning()
    try:
        best = tune.tune(L, X, P, b.cutoff, b.k, reps=1,
                         space_cutoff={"cutoff_wgs_per_cu": [32], **tune.CL_SPAN_CUTOFF},
                         space_knn={"knn_wgs_per_cu": [8], **tune.CL_SPAN_KNN})
        assert set(best["cutoff"]) == {"cutoff_wgs_per_cu", "cutoff_cl_span"}
        assert set(best["knn"]) == {"knn_wgs_per_cu", "knn_cl_span"}
        assert len(best["all"]["cutoff"]) == 2 and len(best["all"]["knn"]) == 2
    finally:
        _lib.set_tuning(**base)
