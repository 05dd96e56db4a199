"""Periodic cutoff and k-nearest-neighbour multigraphs of crystal batches on MI355X.

The compute runs in ``libmatgraph.so`` (hand-written HIP for gfx950 behind a
C ABI declared in ``include/matgraph.h``). This package is the thin Python
binding: it marshals torch tensors (device memory and the current stream)
into the C calls. Importing the package does not load the library; the first
graph call does, and it raises if the library is missing.

Sub-modules:
- ``inputs``: seeded synthetic crystal batches (no method arithmetic);
- ``_lib``:   ctypes loader for ``libmatgraph.so``;
- ``graph``:  ``cutoff_graph``, ``knn_graph``, ``edge_geometry`` and the
              ``EdgeGeometry`` autograd function.
"""

__all__ = ["cutoff_graph", "knn_graph", "edge_geometry", "EdgeGeometry", "Graph"]


def __getattr__(name):
    if name in __all__:
        from . import graph
        return getattr(graph, name)
    raise AttributeError(name)
