"""Seeded graph and edit-stream generators.

The paper evaluates on six public graphs (Wiki, Cora, Flickr, YouTube, Orkut,
Twitter; Sec. 5, dataset table) that are not available here.  These generators
stand in for them with graphs of the same kind: an undirected Erdos-Renyi graph
at Wiki/Cora scale, and directed power-law graphs (Chung-Lu, R-MAT) shaped like
the social graphs (YouTube, Orkut, Twitter).  Every array is a pure function of
the seed.

Edges are returned as ``(src, dst)`` int32 arrays.  Edit batches are
``(src, dst, op)`` with ``op`` = +1 (insert) / -1 (delete) as int8.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "er_undirected",
    "chung_lu_directed",
    "rmat_directed",
    "block_graph",
    "EdgeStream",
    "c1_workload",
    "c2_workload",
    "chung_lu_workload",
    "keys_of",
]


def keys_of(src, dst):
    """64-bit edge keys (src << 32 | dst) used for set membership."""
    return (np.asarray(src, dtype=np.int64) << 32) | np.asarray(dst, dtype=np.int64)


def _distinct_fill(draw, m, rng, undirected):
    """Draw edges with ``draw(count, rng)`` until ``m`` distinct, loop-free ones exist.

    Order of first appearance is kept, so the result is a deterministic
    function of the seed.
    """
    src_parts, dst_parts = [], []
    seen = np.zeros(0, dtype=np.int64)
    have = 0
    while have < m:
        need = m - have
        s, t = draw(int(need * 1.1) + 16, rng)
        if undirected:
            lo, hi = np.minimum(s, t), np.maximum(s, t)
            s, t = lo, hi
        ok = s != t
        s, t = s[ok], t[ok]
        k = keys_of(s, t)
        _, first = np.unique(k, return_index=True)
        first.sort()
        s, t, k = s[first], t[first], k[first]
        fresh = ~np.isin(k, seen)
        s, t, k = s[fresh][:need], t[fresh][:need], k[fresh][:need]
        src_parts.append(s)
        dst_parts.append(t)
        seen = np.concatenate([seen, k])
        have += len(s)
    return (np.concatenate(src_parts).astype(np.int32),
            np.concatenate(dst_parts).astype(np.int32))


def er_undirected(n, m, seed):
    """G(n, m): ``m`` distinct unordered pairs u < v, in random order."""
    rng = np.random.default_rng(seed)

    def draw(c, r):
        return r.integers(0, n, c), r.integers(0, n, c)

    return _distinct_fill(draw, m, rng, undirected=True)


def planted_directed(n, m, blocks, inside, seed):
    """Directed planted-partition graph: ``m`` distinct loop-free edges; with
    probability ``inside`` an edge joins two uniform nodes of one uniform block
    (blocks are contiguous id ranges of n // blocks nodes), else two uniform
    nodes.  Low-rank structure for link-prediction checks."""
    rng = np.random.default_rng(seed)
    size = n // blocks

    def draw(c, r):
        inb = r.random(c) < inside
        b = r.integers(0, blocks, c)
        u = np.where(inb, b * size + r.integers(0, size, c), r.integers(0, n, c))
        v = np.where(inb, b * size + r.integers(0, size, c), r.integers(0, n, c))
        return u, v

    return _distinct_fill(draw, m, rng, undirected=False)


def _chung_lu_weights(n, m, beta):
    """w_i = (i + i0)^(-1/(beta-1)), with i0 chosen so the largest expected degree is sqrt(m)."""
    gamma = 1.0 / (beta - 1.0)
    idx = np.arange(n, dtype=np.float64)

    def top_degree(i0):
        w = (idx + i0) ** (-gamma)
        return m * w[0] / w.sum()

    lo, hi = 1e-3, float(n)
    target = np.sqrt(m)
    for _ in range(200):
        mid = np.sqrt(lo * hi)
        if top_degree(mid) > target:
            lo = mid
        else:
            hi = mid
    w = (idx + hi) ** (-gamma)
    return w / w.sum()


def chung_lu_directed(n, m, beta, seed):
    """Directed Chung-Lu graph with power-law out- and in-weights (exponent ``beta``).

    Out- and in-weights follow the same law with independently permuted labels.
    Self-loops and duplicates are rejected and redrawn.
    """
    rng = np.random.default_rng(seed)
    w = _chung_lu_weights(n, m, beta)
    perm_out = rng.permutation(n)
    perm_in = rng.permutation(n)
    cdf = np.cumsum(w)
    cdf[-1] = 1.0

    def draw(c, r):
        a = np.searchsorted(cdf, r.random(c), side="right")
        b = np.searchsorted(cdf, r.random(c), side="right")
        a = np.minimum(a, n - 1)
        b = np.minimum(b, n - 1)
        return perm_out[a], perm_in[b]

    return _distinct_fill(draw, m, rng, undirected=False)


def rmat_directed(n, m, seed, a=0.57, b=0.19, c=0.19):
    """R-MAT graph on the smallest power of two >= n; ids >= n, loops and duplicates redrawn."""
    rng = np.random.default_rng(seed)
    scale = max(1, int(np.ceil(np.log2(n))))

    def draw(cnt, r):
        s = np.zeros(cnt, dtype=np.int64)
        t = np.zeros(cnt, dtype=np.int64)
        for _ in range(scale):
            x = r.random(cnt)
            right = ((x >= a) & (x < a + b)) | (x >= a + b + c)
            down = x >= a + b
            s = (s << 1) | down
            t = (t << 1) | right
        ok = (s < n) & (t < n)
        return s[ok], t[ok]

    return _distinct_fill(draw, m, rng, undirected=False)


def block_graph(n, blocks, seed, directed=True):
    """Union of ``blocks`` disjoint complete bipartite blocks (rank(A) == blocks).

    Each block is a complete bipartite digraph R_b x C_b on disjoint row and
    column sets, so A is a sum of ``blocks`` rank-1 0/1 matrices with disjoint
    supports.  Used for exactness tests where rank(A) <= d.
    """
    rng = np.random.default_rng(seed)
    perm_r = rng.permutation(n)
    perm_c = rng.permutation(n)
    cuts_r = np.sort(rng.choice(np.arange(1, n), blocks - 1, replace=False))
    cuts_c = np.sort(rng.choice(np.arange(1, n), blocks - 1, replace=False))
    rows = np.split(perm_r, cuts_r)
    cols = np.split(perm_c, cuts_c)
    src, dst = [], []
    for r, c in zip(rows, cols):
        rr, cc = np.meshgrid(r, c, indexing="ij")
        src.append(rr.ravel())
        dst.append(cc.ravel())
    s = np.concatenate(src).astype(np.int32)
    t = np.concatenate(dst).astype(np.int32)
    order = rng.permutation(len(s))
    return s[order], t[order]


class EdgeStream:
    """Edit batches against an evolving directed edge set.

    Inserts pick a uniform source and a destination with probability
    proportional to (in-degree + 1) (preferential attachment), rejecting
    present edges and self-loops.  Deletes pick a uniformly random present
    edge.  Each batch is shuffled.
    """

    def __init__(self, n, src, dst, seed):
        self.n = int(n)
        self.rng = np.random.default_rng(seed)
        keys = keys_of(src, dst)
        order = np.argsort(keys, kind="stable")
        self._init_keys = keys[order]
        self._init_alive = np.ones(len(keys), dtype=bool)
        self._extra = {}  # key -> alive, for keys outside the initial set
        self._edges_src = list(np.asarray(src, dtype=np.int64))
        self._edges_dst = list(np.asarray(dst, dtype=np.int64))
        self._m = len(keys)

    def _lookup(self, key):
        i = int(np.searchsorted(self._init_keys, key))
        if i < len(self._init_keys) and self._init_keys[i] == key:
            return ("init", i)
        return ("extra", key)

    def exists(self, u, v):
        kind, ref = self._lookup((int(u) << 32) | int(v))
        if kind == "init":
            return bool(self._init_alive[ref])
        return self._extra.get(ref, False)

    def _set(self, u, v, alive):
        kind, ref = self._lookup((int(u) << 32) | int(v))
        if kind == "init":
            self._init_alive[ref] = alive
        else:
            self._extra[ref] = alive

    def batch(self, k, insert_frac):
        rng = self.rng
        n = self.n
        n_ins = int(round(k * insert_frac))
        n_del = k - n_ins
        out_s, out_d, out_o = [], [], []
        E = len(self._edges_src)
        for _ in range(n_ins):
            while True:
                u = int(rng.integers(0, n))
                if rng.random() < self._m / (self._m + n):
                    v = int(self._edges_dst[int(rng.integers(0, E))])
                else:
                    v = int(rng.integers(0, n))
                if u != v and not self.exists(u, v):
                    break
            self._set(u, v, True)
            self._edges_src.append(u)
            self._edges_dst.append(v)
            E += 1
            self._m += 1
            out_s.append(u), out_d.append(v), out_o.append(1)
        for _ in range(n_del):
            for _attempt in range(1000):
                j = int(rng.integers(0, E))
                u, v = int(self._edges_src[j]), int(self._edges_dst[j])
                if self.exists(u, v):
                    break
            self._set(u, v, False)
            self._m -= 1
            out_s.append(u), out_d.append(v), out_o.append(-1)
        order = rng.permutation(k)
        return (np.asarray(out_s, dtype=np.int32)[order],
                np.asarray(out_d, dtype=np.int32)[order],
                np.asarray(out_o, dtype=np.int8)[order])


def c1_workload(seed=1, n=2000, m=20000, d=32, batches=200, batch=10):
    """Undirected G(n, m); init on the first 90% of edges; the rest as insert batches."""
    src, dst = er_undirected(n, m, seed)
    n_init = m - batches * batch
    init = (src[:n_init], dst[:n_init])
    stream = []
    for b in range(batches):
        lo = n_init + b * batch
        s = src[lo:lo + batch]
        t = dst[lo:lo + batch]
        stream.append((s.copy(), t.copy(), np.ones(batch, dtype=np.int8)))
    return dict(n=n, d=d, directed=False, init=init, stream=stream,
                alpha=0.15, eps=1e-4)


def chung_lu_workload(n, m, beta, seed, batches, batch, insert_frac, d=128,
                      init_frac=0.9):
    """Directed Chung-Lu graph, init on ``init_frac`` of it, preferential-attachment edits."""
    src, dst = chung_lu_directed(n, m, beta, seed)
    n_init = int(round(m * init_frac))
    init = (src[:n_init].copy(), dst[:n_init].copy())
    stream_gen = EdgeStream(n, init[0], init[1], seed + 1000)
    stream = [stream_gen.batch(batch, insert_frac) for _ in range(batches)]
    heldout = (src[n_init:].copy(), dst[n_init:].copy())
    return dict(n=n, d=d, directed=True, init=init, stream=stream, heldout=heldout)


def c2_workload(seed=2, n=1_000_000, m=10_000_000, batches=1000, batch=1000):
    """Power-law (exponent 2.1) directed graph, d = 128, 95% inserts / 5% deletes."""
    w = chung_lu_workload(n, m, 2.1, seed, batches, batch, 0.95, d=128)
    w.update(alpha=0.15, eps=1e-5, oversample=10, power_iters=2)
    return w
