"""Steps 1-3 as a captured HIP graph (graph_chunks): the same launch sequence
replayed from a graph gives bit-identical results.

Two contexts take the same batches, one launching the chunk kernels one by
one, the other from captured graphs (built on the first batch of each shape,
replayed on later ones, with the library's own eager work -- batch
preparation, graph edits, Step 4, queries -- between the replays).  After
every batch U_b, V_b, P, Sigma and the CSR must agree bit for bit, and the
graph context must report graph launches.
"""
import sys

import numpy as np
import pytest

from workloads import chung_lu_directed

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_graph_replay_bit_identical():
    import torch
    assert torch.cuda.is_available()
    import paper_2306_08967_amd as P
    n, d = 3000, 32
    s0, t0 = chung_lu_directed(n, 30000, 2.1, 19)
    base = dict(directed=True, alpha=0.15, eps=1e-5, max_core_rank=16, max_side=32, tau=1e-6,
                oversample=8, seed=3)
    ca = P.Context.init(P.default_config(n, d, **base), s0, t0)
    cb = P.Context.init(P.default_config(n, d, graph_chunks=8, **base), s0, t0)
    rng = np.random.default_rng(20)
    shapes = set()
    last = None
    for b in range(24):
        k = int(rng.choice([10, 20, 40]))  # a few chunk shapes, each seen several times
        s = rng.integers(0, n, k).astype(np.int32)
        t = rng.integers(0, n, k).astype(np.int32)
        op = np.where(rng.random(k) < 0.2, -1, 1).astype(np.int8)
        ia = ca.update(s, t, op)
        ib = cb.update(s, t, op)
        assert ia["chunks"] == ib["chunks"]
        shapes.add(ib["chunks"])
        last = ib
        xa, xb = ca.export_state(), cb.export_state()
        for key in ("Ub", "Vb", "PU", "PV"):
            assert np.array_equal(xa[key], xb[key]), (b, key)
        assert np.array_equal(ca.singular_values(), cb.singular_values())
        assert np.array_equal(ca.query("Z", np.arange(100, dtype=np.int32)).shape,
                              cb.query("Z", np.arange(100, dtype=np.int32)).shape)
    for tr in (False, True):
        for x, y in zip(ca.export_csr(transpose=tr), cb.export_csr(transpose=tr)):
            assert np.array_equal(x, y)
    _say(f"  chunk counts seen {sorted(shapes)}; graph launches {last['graph_launches']}")
    assert last["graph_launches"] >= 20
    ca.close()
    cb.close()
