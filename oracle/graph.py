"""Graph state and edit semantics (oracle).

The paper models a dynamic graph as a sequence of change events applied to an
initial graph, with A the 0/1 adjacency matrix and D the diagonal out-degree
matrix (Sec. 2, Preliminaries).  An edge change is the update A_t = A_{t-1} +
dA_t with dA = B C^T (Sec. 4.3).  The paper only describes insertions; this
oracle reads a batch of edits as follows (the reading is listed in the design
notes):

* ops are applied in order with set semantics: inserting a present edge and
  deleting an absent edge change nothing;
* for an undirected graph an op on (u, v) edits A[u, v] and A[v, u] together,
  and a self-loop is a single entry;
* the net change of a batch is A_after - A_before, listed as (u, v, +1/-1)
  sorted by (u, v).

Plain Python sets; meant for graphs up to a few million edges.
"""
from __future__ import annotations

import numpy as np


class EdgeSet:
    """Adjacency of a graph as a Python set of (row, col) entries."""

    def __init__(self, n, directed, src=(), dst=()):
        self.n = int(n)
        self.directed = bool(directed)
        self.E = set()
        for u, v in zip(np.asarray(src).tolist(), np.asarray(dst).tolist()):
            self._check(u, v)
            self.E.add((u, v))
            if not self.directed:
                self.E.add((v, u))

    def _check(self, u, v):
        if not (0 <= u < self.n and 0 <= v < self.n):
            raise ValueError(f"edge ({u}, {v}) out of range for n={self.n}")

    def apply(self, src, dst, op):
        """Apply a batch in order; return the net change as a sorted list of (u, v, delta)."""
        before = {}
        for u, v, o in zip(np.asarray(src).tolist(), np.asarray(dst).tolist(),
                           np.asarray(op).tolist()):
            self._check(u, v)
            if o not in (1, -1):
                raise ValueError(f"op must be +1 or -1, got {o}")
            entries = [(u, v)] if (self.directed or u == v) else [(u, v), (v, u)]
            for e in entries:
                if e not in before:
                    before[e] = e in self.E
            if o == 1:
                for e in entries:
                    self.E.add(e)
            else:
                for e in entries:
                    self.E.discard(e)
        net = []
        for e, was in before.items():
            now = e in self.E
            if now != was:
                net.append((e[0], e[1], 1 if now else -1))
        net.sort()
        return net

    def out_degree(self):
        deg = np.zeros(self.n, dtype=np.int64)
        for u, _ in self.E:
            deg[u] += 1
        return deg

    def csr(self, transpose=False):
        """Canonical CSR: int64 indptr, int32 indices ascending within a row, no duplicates."""
        if transpose:
            pairs = sorted((v, u) for (u, v) in self.E)
        else:
            pairs = sorted(self.E)
        indptr = np.zeros(self.n + 1, dtype=np.int64)
        indices = np.empty(len(pairs), dtype=np.int32)
        for i, (r, c) in enumerate(pairs):
            indptr[r + 1] += 1
            indices[i] = c
        np.cumsum(indptr, out=indptr)
        return indptr, indices

    def dense(self):
        A = np.zeros((self.n, self.n), dtype=np.float64)
        for u, v in self.E:
            A[u, v] = 1.0
        return A

    def scipy(self):
        """A as a scipy.sparse CSR matrix of float64 ones."""
        import scipy.sparse as sp
        if not self.E:
            return sp.csr_matrix((self.n, self.n), dtype=np.float64)
        arr = np.array(sorted(self.E), dtype=np.int64)
        data = np.ones(len(arr), dtype=np.float64)
        return sp.csr_matrix((data, (arr[:, 0], arr[:, 1])), shape=(self.n, self.n))

