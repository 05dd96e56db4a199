"""Triplets Gamma_2 of a multigraph (oracle; test infrastructure only).

What is computed (paper Sec. 2.1, Definition def6, third graded component):

    Gamma_2 = {(g, g') in Gamma_1 x Gamma_1 : src(g) = src(g')}

read as ordered pairs of two DIFFERENT edges (the pairs "composed of two edges
sharing the same source", Sec. 2.2, additional functionalities), given as
pairs of edge indices into the graph's edge list. Order: by source, then the
first edge's index, then the second's.

The angle of a triplet is cos(theta) = (v . v') / (|v| |v'|) of the two edge
vectors, 0 when either vector is zero.

Parity status: pinned (closed-form pair counts and angles of small cells,
brute-force enumeration of ordered pairs).
"""
from __future__ import annotations

import numpy as np


def triplets64(row_ptr):
    """(e1, e2) int64 arrays: every ordered pair of distinct edges of one source,
    for a graph whose edges of source i are row_ptr[i] .. row_ptr[i+1]-1."""
    ptr = np.asarray(row_ptr, np.int64)
    e1, e2 = [], []
    for i in range(ptr.shape[0] - 1):
        idx = np.arange(ptr[i], ptr[i + 1], dtype=np.int64)
        d = idx.shape[0]
        a = np.repeat(idx, d)
        b = np.tile(idx, d)
        keep = a != b
        e1.append(a[keep])
        e2.append(b[keep])
    if not e1:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(e1), np.concatenate(e2)


def triplet_cos64(vec, e1, e2):
    """cos(theta) between the edge vectors of every triplet (FP64)."""
    v = np.asarray(vec, np.float64)
    a, b = v[np.asarray(e1, np.int64)], v[np.asarray(e2, np.int64)]
    den = np.sqrt((a * a).sum(1)) * np.sqrt((b * b).sum(1))
    num = (a * b).sum(1)
    return np.where(den > 0.0, num / np.where(den > 0.0, den, 1.0), 0.0)
