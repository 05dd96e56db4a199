"""Helpers for the GPU tests: move seeded batches to the device, run the
library through the Python binding and bring results back as numpy."""
import numpy as np
import torch

from paper_2307_05380_amd import graph, inputs


def dev(batch, device="cuda"):
    return (torch.from_numpy(np.ascontiguousarray(batch.lattices)).to(device),
            torch.from_numpy(np.ascontiguousarray(batch.frac)).to(device),
            torch.from_numpy(np.ascontiguousarray(batch.batch_ptr)).to(device))


def np_graph(g):
    return (g.src.cpu().numpy().astype(np.int64), g.dst.cpu().numpy().astype(np.int64),
            g.image.cpu().numpy().astype(np.int64), g.length.cpu().numpy())


def cutoff(batch, cutoff=None, **kw):  # kw: capacity, image_capacity, strict, opts
    L, X, P = dev(batch)
    g = graph.cutoff_graph(L, X, P, batch.cutoff if cutoff is None else cutoff, **kw)
    torch.cuda.synchronize()
    return g


def knn(batch, k=None, **kw):
    L, X, P = dev(batch)
    g = graph.knn_graph(L, X, P, batch.k if k is None else k, **kw)
    torch.cuda.synchronize()
    return g


def single(L, x, cutoff=5.0, k=8, name="single"):
    L = np.asarray(L, np.float32).reshape(1, 3, 3)
    x = np.asarray(x, np.float32).reshape(-1, 3)
    return inputs.Batch(L, x, np.array([0, x.shape[0]], np.int64), cutoff, k, name)


def concat(batches, cutoff, k):
    lat = np.concatenate([b.lattices for b in batches], 0)
    frac = np.concatenate([b.frac for b in batches], 0)
    ptr = np.zeros(sum(b.B for b in batches) + 1, np.int64)
    ptr[1:] = np.cumsum(np.concatenate([np.diff(b.batch_ptr) for b in batches]))
    return inputs.Batch(lat, frac, ptr, cutoff, k, "concat")
