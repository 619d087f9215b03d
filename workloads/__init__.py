"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only draws graphs and edit streams.  It holds none of the method's
arithmetic (no factorisation, no propagation), so both the oracle and the HIP
path can consume its output without sharing any computation.
"""
from .graphs import (  # noqa: F401
    er_undirected,
    chung_lu_directed,
    rmat_directed,
    block_graph,
    planted_directed,
    EdgeStream,
    c1_workload,
    c2_workload,
    chung_lu_workload,
    keys_of,
)
