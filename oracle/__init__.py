"""FP64 CPU oracle for the periodic cutoff / KNN multigraph and edge geometry.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import, call or
execute this package: it exists so that tests, the smoke check and the
benchmark's CPU-baseline leg can compare the HIP library against a plain,
slow, obviously correct implementation written directly from the paper's
definitions (Sec. 2.1, Definition def6; Sec. 2.2, Algorithms 1 and 2).

It shares no code with the HIP path: it never imports ``paper_2307_05380_amd``
(only test code hands it arrays), and its 3x3 inverse comes from
``numpy.linalg.inv``.

Conventions (also documented in the C header of the library):
- a lattice ``L`` is a 3x3 array whose ROWS are the lattice vectors, so the
  paper's rho is ``L.T`` and an edge vector is ``(x_dst - x_src + t) @ L``;
- an edge is (src, dst, t) with t the integer cell of the destination image;
- the self-image (i, i, 0) is not an edge; (i, i, t != 0) is.

Parity status of every function is listed in ``oracle/graph64.py``,
``oracle/geometry64.py``, ``oracle/triplets64.py`` and ``oracle/symmetrize64.py``; all are pinned by CPU tests (closed forms,
invariants, brute force, finite differences).
"""
from .graph64 import (Graph64, KnnResult64, cutoff_graph64, cutoff_sources64, cutoff_structure64,
                      image_ranges64, knn_graph64, knn_structure64, knn_ties_structure64)
from .symmetrize64 import symmetrize64
from .triplets64 import triplet_cos64, triplets64
from .geometry64 import (edge_geometry64, edge_geometry_vjp64, fd_vjp64, gaussian_loss64,
                         gaussian_loss_grad_len64)

__all__ = [
    "Graph64", "KnnResult64", "cutoff_graph64", "cutoff_sources64", "cutoff_structure64", "image_ranges64",
    "knn_graph64", "knn_structure64", "knn_ties_structure64", "edge_geometry64", "edge_geometry_vjp64", "fd_vjp64",
    "gaussian_loss64", "gaussian_loss_grad_len64", "triplets64", "triplet_cos64",
    "symmetrize64",
]
