"""The allocation-free backward entry point (mg_edge_geometry_backward_static,
scratch in the library's own device array) against mg_edge_geometry_backward
with a caller workspace, through the C ABI: two calls in a row, the second on
a smaller batch (the scratch keeps the first call's contents), both equal to
the workspace call."""
import ctypes

import numpy as np
import pytest
import torch

import gpu_util as gu
from paper_2307_05380_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _case(b, rng):
    g = gu.cutoff(b)
    L, X, P = gu.dev(b)
    E = g.num_edges
    glen = torch.from_numpy(rng.normal(size=E).astype(np.float32)).cuda()
    gvec = torch.from_numpy(rng.normal(size=(E, 3)).astype(np.float32)).cuda()
    return L, X, P, g.src, g.dst, g.image, E, gvec, glen


def _run(lib, B, N, case, static):
    L, X, P, src, dst, image, E, gvec, glen = case
    gf = torch.full((N, 3), float("nan"), dtype=torch.float32, device="cuda")
    gL = torch.full((B, 3, 3), float("nan"), dtype=torch.float32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if static:
        st = lib.mg_edge_geometry_backward_static(_ptr(L), _ptr(X), _ptr(P), B, N, _ptr(src), _ptr(dst), _ptr(image),
                                                  E, None, _ptr(gvec), _ptr(glen), _ptr(gf), _ptr(gL), stream)
    else:
        nbytes = lib.mg_geometry_workspace_bytes(B, N)
        ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")
        st = lib.mg_edge_geometry_backward(_ptr(L), _ptr(X), _ptr(P), B, N, _ptr(src), _ptr(dst), _ptr(image), E,
                                           None, _ptr(gvec), _ptr(glen), _ptr(gf), _ptr(gL), _ptr(ws), ws.numel(),
                                           stream)
    _lib.check(st, lib)
    torch.cuda.synchronize()
    return gf.cpu().numpy(), gL.cpu().numpy()


def test_static_backward_matches_workspace_call():
    lib = _lib.load()
    rng = np.random.default_rng(17)
    big = inputs.make_config2(B=96)
    small = inputs.random_batch(rng, 7, 2, 40, 3.0, 9.0, cutoff=5.0)
    for b in (big, small):   # the second call is smaller than the first
        print(f"static backward: {b.B} structures, {b.N} atoms", flush=True)
        case = _case(b, rng)
        gf_s, gL_s = _run(lib, b.B, b.N, case, static=True)
        gf_w, gL_w = _run(lib, b.B, b.N, case, static=False)
        assert np.isfinite(gf_s).all() and np.isfinite(gL_s).all()
        tol_f = 1e-5 * max(np.abs(gf_w).max(), 1e-30)
        tol_L = 1e-5 * max(np.abs(gL_w).max(), 1e-30)
        assert np.abs(gf_s - gf_w).max() <= tol_f
        assert np.abs(gL_s - gL_w).max() <= tol_L


def test_static_backward_rejects_batches_beyond_the_scratch():
    lib = _lib.load()
    fake = ctypes.c_void_p(16)
    N = 1 << 23   # needs more than the 16 MiB of static scratch
    st = lib.mg_edge_geometry_backward_static(fake, fake, fake, 1, N, fake, fake, fake, 0, None, None, None,
                                              None, None, None)
    assert st == _lib.MG_ERR_UNSUPPORTED
    assert b"static scratch" in lib.mg_last_error()
