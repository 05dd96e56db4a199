"""Symmetric closure of a multigraph (oracle; test infrastructure only).

What is computed (paper Sec. 2.2, additional functionalities: a procedure that
makes a directed graph symmetric by adding the missing edges, each edge once):

    S = E  union  {(j, i, -t) : (i, j, t) in E}

for an edge list E grouped by source (row_ptr) whose edges are unique. The
reverse of an edge has the same length (||(x_i - x_j - t) L|| = ||(x_j - x_i + t) L||).

Order (a reading; the paper fixes none): source by source, first the source's
own input edges in their input order, then the reverse edges it receives that
were missing, ordered by the index of the input edge they reverse.

Parity status: pinned (closed-form KNN chain, symmetry, set identity,
idempotence, symmetric inputs unchanged).
"""
from __future__ import annotations

import numpy as np


def symmetrize64(row_ptr, dst, image, length=None):
    """Returns (row_ptr [N+1], src, dst, image [S,3], length or None) of S."""
    ptr = np.asarray(row_ptr, np.int64)
    dst = np.asarray(dst, np.int64)
    img = np.asarray(image, np.int64).reshape(-1, 3)
    N = ptr.shape[0] - 1
    src = np.repeat(np.arange(N, dtype=np.int64), np.diff(ptr))
    present = {(int(a), int(b), int(t[0]), int(t[1]), int(t[2])) for a, b, t in zip(src, dst, img)}
    incoming = [[] for _ in range(N)]          # reversed input edges that are missing, by target
    for e in range(src.shape[0]):
        i, j, t = int(src[e]), int(dst[e]), img[e]
        if (j, i, -int(t[0]), -int(t[1]), -int(t[2])) not in present:
            incoming[j].append(e)
    out_src, out_dst, out_img, out_len, out_ptr = [], [], [], [], [0]
    for i in range(N):
        own = range(ptr[i], ptr[i + 1])
        for e in own:
            out_src.append(i)
            out_dst.append(int(dst[e]))
            out_img.append(img[e])
            out_len.append(None if length is None else length[e])
        for e in incoming[i]:                  # already in input-edge order
            out_src.append(i)
            out_dst.append(int(src[e]))
            out_img.append(-img[e])
            out_len.append(None if length is None else length[e])
        out_ptr.append(len(out_src))
    S = len(out_src)
    return (np.asarray(out_ptr, np.int64), np.asarray(out_src, np.int64).reshape(S),
            np.asarray(out_dst, np.int64).reshape(S), np.asarray(out_img, np.int64).reshape(S, 3),
            None if length is None else np.asarray(out_len, np.asarray(length).dtype).reshape(S))
