"""DAMF driver in explicit form (oracle).

Algorithm 2 (edge branch) per batch: turn the events into B, C, apply
UpdateEmbeddingE, update the embeddings, then refresh the enhanced embedding
(Step 4).  Appendix A (Algorithm 3) initialises from a t-SVD of A.  The query
returns rows of X = U Sigma^(1/2), Y = V Sigma^(1/2) (Sec. 4.1) and of the
enhanced context embedding Z = PPR(X) (Sec. 4.4), which by linearity of PPR is
PPR(U) Sigma^(1/2).

This driver keeps U and V explicitly (the lazy base space of Sec. 4.1 is an
implementation device that does not change the result in exact arithmetic),
and recomputes Z from the PPR series on every query, so its Z is the exact
PPR of the current X.
"""
from __future__ import annotations

import numpy as np

from . import factor, node, ppr, update
from .graph import EdgeSet


class DAMFOracle:
    def __init__(self, n, d, directed, alpha=0.15, eps=1e-4, r=32, r_max=64, tau=1e-6):
        self.n, self.d = int(n), int(d)
        self.directed = bool(directed)
        self.alpha, self.eps = float(alpha), float(eps)
        self.r, self.r_max, self.tau = int(r), int(r_max), float(tau)
        self.graph = None
        self.U = self.s = self.V = None

    # ---- initialisation (Appendix A, Algorithm 3)
    def init_exact(self, src, dst):
        self.graph = EdgeSet(self.n, self.directed, src, dst)
        self.U, self.s, self.V = factor.tsvd_exact(self.graph.dense(), self.d)
        return self

    def init_randomized(self, src, dst, oversample, power_iters, seed):
        self.graph = EdgeSet(self.n, self.directed, src, dst)
        A = self.graph.scipy()
        self.U, self.s, self.V = factor.tsvd_randomized(A, self.d, oversample, power_iters, seed)
        return self

    def init_factors(self, src, dst, U, s, V):
        self.graph = EdgeSet(self.n, self.directed, src, dst)
        self.U = np.array(U, dtype=np.float64)
        self.s = np.array(s, dtype=np.float64)
        self.V = np.array(V, dtype=np.float64)
        return self

    # ---- one batch (Algorithm 2, edge branch; Algorithm 1 per chunk)
    def update(self, src, dst, op):
        net = self.graph.apply(src, dst, op)
        chunks = update.chunk(net, self.directed, self.r, self.r_max)
        infos = []
        for (S1, S2, D) in chunks:
            self.U, self.s, self.V, info = update.chunk_update(
                self.U, self.s, self.V, S1, S2, D, self.tau)
            infos.append(dict(s1=len(S1), s2=len(S2), rho_b=info["rho_b"], rho_c=info["rho_c"]))
        return dict(net=net, chunks=chunks, chunk_info=infos)

    # ---- node change (Algorithm 2, node branch; Theorem 1)
    def add_node(self, new, in_nbrs, out_nbrs=()):
        """Node `new`, without edges so far, joins with in-edges (v, new) and
        out-edges (new, w) (undirected: the neighbours in in_nbrs): the graph
        gains the edges, and the factorisation takes Theorem 1's column step
        then its row step, each cut into pieces of at most r_max entries."""
        if any(u == new or v == new for (u, v) in self.graph.E):
            raise ValueError("node change needs a node without edges")
        ins = [int(v) for v in in_nbrs]
        outs = ins if not self.directed else [int(w) for w in out_nbrs]
        if self.directed:
            src = [v for v in ins] + [new] * len(outs)
            dst = [new] * len(ins) + outs
        else:
            src, dst = [new] * len(ins), ins
        self.graph.apply(np.array(src, dtype=np.int64), np.array(dst, dtype=np.int64),
                         np.ones(len(src), dtype=np.int64))
        self.U, self.s, self.V, info = node.node_event(self.U, self.s, self.V, new, ins, outs,
                                                       self.tau, self.r_max)
        return info

    # ---- query (Sec. 4.1 and Sec. 4.4)
    def X(self):
        return self.U * np.sqrt(self.s)[None, :]

    def Y(self):
        return self.V * np.sqrt(self.s)[None, :]

    def Z(self):
        return ppr.ppr_series(self.graph.scipy(), self.U, self.alpha) * np.sqrt(self.s)[None, :]

    def query(self, which, nodes=None):
        M = {"X": self.X, "Y": self.Y, "Z": self.Z}[which]()
        return M if nodes is None else M[np.asarray(nodes)]
