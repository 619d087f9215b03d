"""The paper-faithful single-edit mode (Sec. 4.3 treats one edge at a time:
Theorem 2 with n x 1 B and C, a (d+1) x (d+1) core per edge; Algorithm 1
UpdateEmbeddingE).  With chunk rank r = r_max = 1 every directed edit is its
own chunk, so the library runs exactly the paper's per-edge sequence.

1. Parity: a directed stream applied with r = r_max = 1 on the GPU against the
   oracle with the same chunking (one edge per update): singular values
   within 1e-5 s_1, X Y^T within 1e-5 relative Frobenius error,
   orthonormality 1e-5; every chunk had one edit and a core of d + 1 at most.
2. Effect of the chunk rank: the same stream applied in chunks of rank <= 16
   and edit by edit; both are compared with the exact rank-d t-SVD of the
   final graph (relative reconstruction error ||A - X Y^T||_F / ||A||_F and
   the product distance), reported, and the batched form must be as close to
   the exact t-SVD as the edit-by-edit form up to 1e-3 relative.
"""
import sys

import numpy as np
import pytest

from oracle.factor import tsvd_exact
from oracle.model import DAMFOracle
from tests._checks import orth_err, product_rel_err, recon_err2, unit_factor
from workloads import chung_lu_directed

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def damf():
    import torch
    assert torch.cuda.is_available()
    import paper_2306_08967_amd as P
    P.lib()
    return P


def _stream(n, m, seed, batches, k):
    s0, t0 = chung_lu_directed(n, m, 2.1, seed)
    n_init = int(0.8 * m)
    init = (s0[:n_init], t0[:n_init])
    rest = (s0[n_init:], t0[n_init:])
    out = []
    for b in range(batches):
        s, t = rest[0][b * k:(b + 1) * k], rest[1][b * k:(b + 1) * k]
        out.append((s, t, np.ones(len(s), np.int8)))
    return init, out


def test_single_edit_parity(damf):
    n, m, d = 600, 6000, 16
    _say("case k=1 parity")
    init, stream = _stream(n, m, 91, 20, 10)
    orc = DAMFOracle(n, d, True, alpha=1.0, r=1, r_max=1, tau=1e-6).init_exact(*init)
    cfg = damf.default_config(n, d, directed=True, alpha=1.0, max_core_rank=1, max_side=1, tau=1e-6)
    ctx = damf.Context.init_factors(cfg, init[0], init[1], orc.U, orc.s, orc.V)
    for s, t, op in stream:
        io = orc.update(s, t, op)
        info = ctx.update(s, t, op)
        assert info["chunks"] == len(io["net"])  # one chunk per edit
        assert info["max_core"] <= d + 1
    sg = ctx.singular_values()
    X, Y = ctx.query("X"), ctx.query("Y")
    err_s = np.abs(sg - orc.s).max() / orc.s[0]
    err_p = product_rel_err(X, Y, orc.X(), orc.Y())
    eo = max(orth_err(unit_factor(X, sg)), orth_err(unit_factor(Y, sg)))
    _say(f"  sigma {err_s:.2e} product {err_p:.2e} orth {eo:.2e}")
    assert err_s <= 1e-5 and err_p <= 1e-5 and eo <= 1e-5
    ctx.close()


def test_chunk_rank_against_single_edits(damf):
    n, m, d = 1500, 20000, 32
    _say("case chunk rank vs k=1")
    init, stream = _stream(n, m, 92, 40, 100)
    U, s, V = tsvd_exact(_dense(n, *init), d)
    res = {}
    for r in (1, 16):
        cfg = damf.default_config(n, d, directed=True, alpha=1.0, max_core_rank=r, max_side=max(r, 1),
                                  tau=1e-6)
        ctx = damf.Context.init_factors(cfg, init[0], init[1], U, s, V)
        chunks = 0
        for a, b, op in stream:
            chunks += ctx.update(a, b, op)["chunks"]
        res[r] = (ctx.query("X").astype(np.float64), ctx.query("Y").astype(np.float64), chunks)
        ctx.close()
    src = np.concatenate([init[0]] + [b[0] for b in stream])
    dst = np.concatenate([init[1]] + [b[1] for b in stream])
    A = _dense(n, src, dst)
    Ue, se, Ve = tsvd_exact(A, d)
    import scipy.sparse as sp
    As = sp.csr_matrix(A)
    nA = np.sqrt(As.nnz)
    rec_exact = np.sqrt(max(recon_err2(As, Ue * np.sqrt(se), Ve * np.sqrt(se)), 0.0)) / nA
    out = {}
    for r, (X, Y, chunks) in res.items():
        rec = np.sqrt(max(recon_err2(As, X, Y), 0.0)) / nA
        dist = product_rel_err(X, Y, Ue * np.sqrt(se), Ve * np.sqrt(se))
        out[r] = (rec, dist)
        _say(f"  r={r}: {chunks} chunks, reconstruction {rec:.6f} (exact t-SVD {rec_exact:.6f}), "
             f"product distance to the exact t-SVD {dist:.3e}")
    between = product_rel_err(res[16][0], res[16][1], res[1][0], res[1][1])
    _say(f"  product distance between r=16 and r=1: {between:.3e}")
    assert out[16][0] <= out[1][0] * (1 + 1e-3)
    assert out[1][0] >= rec_exact * (1 - 1e-9) and out[16][0] >= rec_exact * (1 - 1e-9)


def _dense(n, src, dst):
    A = np.zeros((n, n))
    A[np.asarray(src), np.asarray(dst)] = 1.0
    return A
