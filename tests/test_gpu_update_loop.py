"""The 64-supercell update workload on the GPU (cell lists): 100 steps of
Cartesian N(0, 0.02 A) moves, each rebuilding the cutoff graph (5 A, with edge
vectors from the fill) and the KNN graph (k = 32) and running the geometry
backward pass, as a model that moves atoms inside its forward pass would
(abstract; Sec. 4). After the moves of steps 0, 50 and 99 the graphs and the
gradients are checked against the FP64 oracle on the moved coordinates:
cutoff rows and KNN rows of sampled sources of every supercell (Definition
def6 and the k-nearest rule, band rule as for every graph test), coordinate
gradients of sampled atoms (every edge that touches them) and the lattice
gradients of two supercells (all their edges)."""
import numpy as np
import pytest
import torch

import compare
import oracle
from paper_2307_05380_amd import _lib, graph, inputs

pytestmark = pytest.mark.gpu

CHECKED = (0, 50, 99)
SOURCES_PER_SUPERCELL = 8


def _sample(n, count, seed):
    return sorted(np.random.default_rng(seed).choice(n, min(count, n), replace=False).tolist())


def _rel(a, ref, scale):
    return float(np.abs(np.asarray(a, np.float64) - ref).max() / max(scale, 1e-300))


def test_update_loop_parity_steps_0_50_99():
    b = inputs.make_config5()
    dev = torch.device("cuda")
    L = torch.from_numpy(b.lattices).to(dev)
    X = torch.from_numpy(b.frac).to(dev)
    P = torch.from_numpy(b.batch_ptr).to(dev)
    E0, icap = graph.cutoff_sizes(L, X, P, b.cutoff)
    cap = int(E0 * 1.15) + 4096
    cb = graph.CutoffBuilder(b.B, b.N, cap, max(icap, 4096), dev, vec=True)
    kb = graph.KnnBuilder(b.B, b.N, b.k, 4096, dev)
    geo = graph.GeometryRunner(b.B, b.N, dev)
    glen = torch.from_numpy(np.random.default_rng(5).normal(size=cap).astype(np.float32)).to(dev)
    gf = torch.empty_like(X)
    gL = torch.empty_like(L)
    ne = cb.rep[:1]
    for step in range(max(CHECKED) + 1):
        X.add_(torch.from_numpy(inputs.config5_step_delta(b, step)).to(dev))
        cb.run(L, X, P, b.cutoff, 0)
        kb.run(L, X, P, 0)
        geo.backward(L, X, P, cb.src, cb.dst, cb.image, None, glen, gf, gL, num_edges=ne)
        if step not in CHECKED:
            continue
        torch.cuda.synchronize()
        rc, rk = cb.report(), kb.report()
        print(f"step {step}: {rc.num_edges} cutoff edges, flags 0x{rc.flags:x} / 0x{rk.flags:x}", flush=True)
        assert rc.flags == 0, rc.flag_names()
        assert rk.flags & ~_lib.MG_FLAG_KNN_EXTENDED == 0, rk.flag_names()
        E = rc.num_edges
        moved = inputs.Batch(b.lattices, X.cpu().numpy(), b.batch_ptr, b.cutoff, b.k, f"config5 step {step}")
        rp = cb.row_ptr.cpu().numpy()
        assert rp[-1] == E
        k_dst = kb.dst.cpu().numpy()
        k_img = kb.image.cpu().numpy()
        k_len = kb.length.cpu().numpy()
        near = 0
        for q in range(b.B):
            a0, a1 = int(b.batch_ptr[q]), int(b.batch_ptr[q + 1])
            srcs = _sample(a1 - a0, SOURCES_PER_SUPERCELL, 1000 * step + q)
            rows = np.concatenate([np.arange(rp[a0 + i], rp[a0 + i + 1]) for i in srcs])
            idx = torch.from_numpy(rows).to(dev)
            s = cb.src[idx].cpu().numpy().astype(np.int64)
            d = cb.dst[idx].cpu().numpy().astype(np.int64)
            t = cb.image[idx].cpu().numpy().astype(np.int64)
            ln = cb.length[idx].cpu().numpy()
            st = compare.cutoff_sources_check(moved, q, srcs, s, d, t, ln)
            near += st["near"]
            # edge vectors from the fill against the FP64 geometry
            v64, _ = oracle.edge_geometry64(b.lattices, moved.frac, b.batch_ptr, s, d, t)
            assert np.abs(cb.vec[idx].cpu().numpy() - v64).max() <= compare.LEN_TOL
            compare.knn_sources_check(moved, q, b.k, srcs, None, k_dst, k_img, k_len)
        print(f"step {step}: cutoff and KNN rows of {SOURCES_PER_SUPERCELL} sources per supercell match, "
              f"{near} cutoff candidates inside the band", flush=True)
        # coordinate gradients of sampled atoms: every edge with the atom as src or dst
        atoms = np.sort(np.concatenate([int(b.batch_ptr[q]) + np.array(_sample(int(b.batch_ptr[q + 1] - b.batch_ptr[q]),
                                                                                 1, 77 + step + q))
                                        for q in range(0, b.B, 4)]))
        at = torch.from_numpy(atoms.astype(np.int32)).to(dev)
        touch = torch.nonzero(torch.isin(cb.src[:E], at) | torch.isin(cb.dst[:E], at)).flatten()
        s = cb.src[touch].cpu().numpy().astype(np.int64)
        d = cb.dst[touch].cpu().numpy().astype(np.int64)
        t = cb.image[touch].cpu().numpy().astype(np.int64)
        g = glen[touch].cpu().numpy()
        rf, _ = oracle.edge_geometry_vjp64(b.lattices, moved.frac, b.batch_ptr, s, d, t, None, g)
        got = gf.cpu().numpy()
        scale = np.abs(rf[atoms]).max()
        err = _rel(got[atoms], rf[atoms], scale)
        # lattice gradients of two supercells (all their edges)
        for q in (step % b.B, (step + 31) % b.B):
            e0, e1 = int(rp[b.batch_ptr[q]]), int(rp[b.batch_ptr[q + 1]])
            s = cb.src[e0:e1].cpu().numpy().astype(np.int64)
            d = cb.dst[e0:e1].cpu().numpy().astype(np.int64)
            t = cb.image[e0:e1].cpu().numpy().astype(np.int64)
            g = glen[e0:e1].cpu().numpy()
            _, rL = oracle.edge_geometry_vjp64(b.lattices, moved.frac, b.batch_ptr, s, d, t, None, g)
            err = max(err, _rel(gL[q].cpu().numpy(), rL[q], np.abs(rL[q]).max()))
        print(f"step {step}: gradient relative error {err:.3g}", flush=True)
        assert err <= 1e-4
