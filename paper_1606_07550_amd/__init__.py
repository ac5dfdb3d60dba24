"""Exact triangle counting and clustering coefficients on MI355X (gfx950).

The operation is SNAP's triadic-closure analytics (node clustering
coefficient and triangle counting) on an undirected simple graph held as
sorted per-node adjacency lists. The native library ``libtricc.so`` (HIP
kernels + C ABI, ``include/tricc.h``) does all the work; this package only
marshals arguments. Importing it does not load the library; the first call
that needs it does, and raises if it is not built.
"""
from .graph import Graph, count, default_tuning, variant_capacity, variant_count, workspace_size  # noqa: F401
from ._native import TriccError  # noqa: F401
from .batch import Batch, batch_workspace_size, default_batch_tuning  # noqa: F401
from .serve import Server  # noqa: F401
from . import generators  # noqa: F401
