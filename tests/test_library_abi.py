"""The C-ABI library loads, exports every symbol include/matgraph.h declares,
and validates arguments on the host (CPU only: no compute call reaches a GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "matgraph.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2307_05380_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2307_05380_amd.build import build
        build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    from paper_2307_05380_amd import _lib
    names = _declared()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (mg_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(names) == set(_lib.SIGNATURES), "binding signatures and header disagree"
    for n in names:
        assert hasattr(lib, n)


def test_abi_version_and_sizes(lib):
    assert lib.mg_abi_version() == 1
    a = lib.mg_cutoff_workspace_bytes(10, 100, 0)
    b = lib.mg_cutoff_workspace_bytes(10, 100, 1000)
    assert a > 0 and b - a == 45 * 1000   # per image slot: box entry, flag, scan value, kept entry
    assert lib.mg_cutoff_workspace_bytes(-1, 10, 0) == 0
    assert lib.mg_knn_workspace_bytes(10, 100, 0, 10) == 0
    assert lib.mg_knn_workspace_bytes(10, 100, 65, 10) == 0
    assert lib.mg_knn_workspace_bytes(10, 100, 16, 10) > 0
    assert lib.mg_geometry_workspace_bytes(4, 10) >= 4 * 10 + 9 * 8 * 4


def _cutoff(lib, **kw):
    P = ctypes.c_void_p
    fake = P(0x1000)
    args = dict(lattices=fake, frac=fake, ptr=fake, B=1, N=2, cutoff=3.0, capacity=0, src=None, dst=None,
                image=None, length=None, row_ptr=None, report=fake, ws=fake, wsb=1 << 20, opts=0, stream=None)
    args.update(kw)
    return lib.mg_cutoff_graph(*args.values())


def test_host_validation(lib):
    from paper_2307_05380_amd import _lib
    assert _cutoff(lib, B=-1) == _lib.MG_ERR_INVALID_ARG
    assert b"B must be" in lib.mg_last_error()
    assert _cutoff(lib, cutoff=0.0) == _lib.MG_ERR_INVALID_ARG
    assert _cutoff(lib, cutoff=float("nan")) == _lib.MG_ERR_INVALID_ARG
    assert _cutoff(lib, capacity=5) == _lib.MG_ERR_INVALID_ARG       # outputs NULL with capacity > 0
    assert _cutoff(lib, report=None) == _lib.MG_ERR_INVALID_ARG
    assert _cutoff(lib, ws=None) == _lib.MG_ERR_WORKSPACE
    assert _cutoff(lib, wsb=16) == _lib.MG_ERR_WORKSPACE
    assert _cutoff(lib, ptr=None) == _lib.MG_ERR_INVALID_ARG
    assert _cutoff(lib, B=0, N=3) == _lib.MG_ERR_INVALID_ARG
    assert _cutoff(lib, opts=1 << 10) == _lib.MG_ERR_INVALID_ARG
    P = ctypes.c_void_p
    fake = P(0x1000)
    st = lib.mg_knn_graph(fake, fake, fake, 1, 2, 0, fake, fake, fake, fake, fake, fake, 1 << 20, 0, None)
    assert st == _lib.MG_ERR_INVALID_ARG and b"k must be" in lib.mg_last_error()
    st = lib.mg_edge_geometry(fake, fake, fake, 1, 2, None, None, None, 5, None, None, None, fake, 1 << 20, None)
    assert st == _lib.MG_ERR_INVALID_ARG


def test_host_validation_extra_entry_points(lib):
    """Argument checks of the per-atom-cutoff, keep-ties, symmetrisation and
    triplet calls (all rejected on the host, before any device work)."""
    from paper_2307_05380_amd import _lib
    P = ctypes.c_void_p
    fake = P(0x1000)
    ERR, WS = _lib.MG_ERR_INVALID_ARG, _lib.MG_ERR_WORKSPACE
    # per-atom cutoffs: radii NULL with atoms
    st = lib.mg_cutoff_graph_radii(fake, fake, fake, 1, 2, None, 0, None, None, None, None, None, fake, fake,
                                   1 << 20, 0, None)
    assert st == ERR and b"radii" in lib.mg_last_error()
    # cutoff graph with edge vectors: vec NULL with capacity, then the cutoff checks of the plain call
    st = lib.mg_cutoff_graph_vec(fake, fake, fake, 1, 2, 5.0, None, 8, fake, fake, fake, fake, None, None, fake,
                                 fake, 1 << 20, 0, None)
    assert st == ERR and b"vec" in lib.mg_last_error()
    st = lib.mg_cutoff_graph_vec(fake, fake, fake, 1, 2, -1.0, None, 0, None, None, None, None, None, None, fake,
                                 fake, 1 << 20, 0, None)
    assert st == ERR and b"cutoff" in lib.mg_last_error()
    # keep-ties KNN: k outside 1..63, NULL outputs with capacity, NULL workspace
    for k in (0, 64):
        st = lib.mg_knn_graph_ties(fake, fake, fake, 1, 2, k, 0, None, None, None, None, None, fake, fake,
                                   1 << 20, 0, None)
        assert st == ERR and b"k must be" in lib.mg_last_error()
    st = lib.mg_knn_graph_ties(fake, fake, fake, 1, 2, 4, 8, None, None, None, None, None, fake, fake, 1 << 20,
                               0, None)
    assert st == ERR
    st = lib.mg_knn_graph_ties(fake, fake, fake, 1, 2, 4, 0, None, None, None, None, None, fake, None, 0, 0, None)
    assert st == WS
    assert lib.mg_knn_ties_workspace_bytes(2, 10, 64, 0) == 0
    assert lib.mg_knn_ties_workspace_bytes(2, 10, 16, 0) > lib.mg_knn_workspace_bytes(2, 10, 64, 0)
    # symmetrisation: NULL row_ptr, NULL edges, out_length without lengths, small workspace
    st = lib.mg_symmetrize(None, 2, fake, fake, None, 4, 0, None, None, None, None, None, fake, fake, 1 << 20, None)
    assert st == ERR and b"row_ptr" in lib.mg_last_error()
    st = lib.mg_symmetrize(fake, 2, None, None, None, 4, 0, None, None, None, None, None, fake, fake, 1 << 20, None)
    assert st == ERR
    st = lib.mg_symmetrize(fake, 2, fake, fake, None, 4, 8, fake, fake, fake, fake, None, fake, fake, 1 << 20, None)
    assert st == ERR and b"out_length" in lib.mg_last_error()
    st = lib.mg_symmetrize(fake, 2, fake, fake, None, 4, 0, None, None, None, None, None, fake, fake, 8, None)
    assert st == WS
    assert lib.mg_symmetrize_workspace_bytes(-1, 4) == 0
    # triplets: E beyond int32, cos without vectors, NULL outputs with capacity
    st = lib.mg_triplets(fake, 2, 1 << 31, None, 0, None, None, None, None, fake, fake, 1 << 20, None)
    assert st == ERR
    st = lib.mg_triplets(fake, 2, 4, None, 8, fake, fake, fake, None, fake, fake, 1 << 20, None)
    assert st == ERR and b"vec" in lib.mg_last_error()
    st = lib.mg_triplets(fake, 2, 4, None, 8, None, None, None, None, fake, fake, 1 << 20, None)
    assert st == ERR
    assert lib.mg_triplets_workspace_bytes(-1) == 0 and lib.mg_triplets_workspace_bytes(10) > 0


def test_host_validation_images_needed(lib):
    """The image-table sizing query rejects bad k, bad cutoffs and a missing
    report or workspace on the host."""
    from paper_2307_05380_amd import _lib
    P = ctypes.c_void_p
    fake = P(0x1000)
    ERR, WS = _lib.MG_ERR_INVALID_ARG, _lib.MG_ERR_WORKSPACE
    for k in (-1, 65):
        st = lib.mg_images_needed(fake, fake, fake, 1, 2, 5.0, None, k, fake, fake, 1 << 20, 0, None)
        assert st == ERR and b"k must be" in lib.mg_last_error()
    st = lib.mg_images_needed(fake, fake, fake, 1, 2, 0.0, None, 0, fake, fake, 1 << 20, 0, None)
    assert st == ERR and b"cutoff" in lib.mg_last_error()
    st = lib.mg_images_needed(fake, fake, fake, 1, 2, 5.0, None, 0, None, fake, 1 << 20, 0, None)
    assert st == ERR and b"report" in lib.mg_last_error()
    st = lib.mg_images_needed(fake, fake, fake, 1, 2, 5.0, None, 4, fake, None, 0, 0, None)
    assert st == WS
    st = lib.mg_images_needed(fake, fake, fake, 1, 2, 5.0, None, 4, fake, fake, 16, 0, None)
    assert st == WS


def test_tuning_roundtrip(lib):
    from paper_2307_05380_amd import _lib
    t0 = _lib.get_tuning()
    assert t0["cutoff_slots"] in (1, 2, 4)
    with pytest.raises(_lib.MatgraphError):
        _lib.set_tuning(cutoff_slots=3)
    _lib.set_tuning(cutoff_slots=4)
    assert _lib.get_tuning()["cutoff_slots"] == 4
    _lib.set_tuning(**{k: v for k, v in t0.items()})
    assert _lib.get_tuning() == t0
    assert _lib.profile_read() == {}
