"""Link scores (damf_score_pairs) and the synthetic link-prediction /
reconstruction harness (Sec. 5.2 tasks; the appendix's scoring rule).

1. Kernel parity: scores <A[u], B[v]> equal the FP64 dot products of the
   GPU's own queried rows (1e-5 relative to the score scale); with X and Y
   they match the oracle's (X Y^T)[u, v] within 1e-5 of max |X_o Y_o^T|;
   DAMF_SCORE_BOTH_WAYS gives the larger of both directions.
2. Quality: a planted-partition graph loses 30% of its edges; the rest is
   embedded by a randomized init on half of it plus streamed updates of the
   other half (the dynamic path), and by a static randomized t-SVD of all of
   it (the oracle).  Held-out edges against as many non-edges are scored by
   <Z[u], Y[v]>; the dynamic AUC and AP must be high (> 0.9) and within 0.02
   of the static embedding's; precision@K of graph reconstruction is reported
   on a 1% pair sample.
"""
import sys

import numpy as np
import pytest

from oracle.factor import tsvd_randomized
from oracle.model import DAMFOracle
from oracle.ppr import ppr_series
from workloads import c1_workload, planted_directed
from workloads import linkpred as lp

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


def test_score_pairs_kernel(damf):
    import torch
    _say("case score pairs kernel")
    w = c1_workload()
    n, d = w["n"], w["d"]
    orc = DAMFOracle(n, d, False, alpha=0.15, eps=1e-4, r=32, r_max=64,
                     tau=1e-6).init_exact(*w["init"])
    cfg = damf.default_config(n, d, directed=False, alpha=0.15, eps=1e-4, max_core_rank=32,
                              max_side=64, tau=1e-6)
    ctx = damf.Context.init_factors(cfg, w["init"][0], w["init"][1], orc.U, orc.s, orc.V)
    for s, t, op in w["stream"][:30]:
        orc.update(s, t, op)
        ctx.update(s, t, op)
    rng = np.random.default_rng(5)
    u = rng.integers(0, n, 5000).astype(np.int32)
    v = rng.integers(0, n, 5000).astype(np.int32)
    Z, Y, X = (ctx.query(k).astype(np.float64) for k in ("Z", "Y", "X"))
    ref = np.einsum("ij,ij->i", Z[u], Y[v])
    got = ctx.score_pairs(u, v, "Z", "Y")
    scale = np.abs(ref).max()
    _say(f"  Z.Y vs own rows: {np.abs(got - ref).max() / scale:.2e}")
    assert np.abs(got - ref).max() <= 1e-5 * scale
    both = ctx.score_pairs(u, v, "Z", "Y", both_ways=True)
    ref2 = np.maximum(ref, np.einsum("ij,ij->i", Z[v], Y[u]))
    assert np.abs(both - ref2).max() <= 1e-5 * scale
    dev = ctx.score_pairs(torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda(), "Z", "Y")
    assert np.array_equal(dev.cpu().numpy(), got)
    # X, Y against the oracle's product entries
    Po = orc.X() @ orc.Y().T
    gxy = ctx.score_pairs(u, v, "X", "Y")
    err = np.abs(gxy - Po[u, v]).max() / np.abs(Po).max()
    _say(f"  X.Y vs oracle entries: {err:.2e}")
    assert err <= 1e-5
    with pytest.raises(damf.DamfError):
        ctx.score_pairs(np.array([0, n], np.int32), np.array([1, 2], np.int32))
    ctx.close()


def test_link_prediction_quality(damf):
    n, m, blocks, d = 4000, 60_000, 16, 32
    alpha, eps = 0.15, 1e-5
    _say(f"case link prediction n={n} m={m} planted blocks={blocks} d={d}")
    src, dst = planted_directed(n, m, blocks, 0.95, seed=81)
    (ks, kt), (rs, rt) = lp.holdout_split(src, dst, 0.3, seed=82)
    keys = lp.edge_keys(src, dst, n)
    nu, nv = lp.negative_pairs(n, len(rs), keys, seed=83)
    half = len(ks) // 2
    cfg = damf.default_config(n, d, directed=True, alpha=alpha, eps=eps, oversample=10,
                              power_iters=2, seed=7, max_core_rank=32, max_side=64)
    ctx = damf.Context.init(cfg, ks[:half], kt[:half])
    for i in range(half, len(ks), 500):
        s, t = ks[i:i + 500], kt[i:i + 500]
        ctx.update(s, t, np.ones(len(s), np.int8))
    pos = ctx.score_pairs(rs.astype(np.int32), rt.astype(np.int32), "Z", "Y")
    neg = ctx.score_pairs(nu, nv, "Z", "Y")
    auc_d, ap_d = lp.auc(pos, neg), lp.average_precision(pos, neg)
    # static reference: the oracle's randomized t-SVD of the same kept graph
    import scipy.sparse as sp
    A = sp.csr_matrix((np.ones(len(ks)), (ks, kt)), shape=(n, n))
    U, s, V = tsvd_randomized(A, d, 10, 2, 7)
    Zs = ppr_series(A, U, alpha) * np.sqrt(s)
    Ys = V * np.sqrt(s)
    pos_s = np.einsum("ij,ij->i", Zs[rs], Ys[rt])
    neg_s = np.einsum("ij,ij->i", Zs[nu], Ys[nv])
    auc_s, ap_s = lp.auc(pos_s, neg_s), lp.average_precision(pos_s, neg_s)
    # reconstruction on a 1% sample of all ordered pairs of the full graph
    rng = np.random.default_rng(84)
    q = n * n // 100
    pu = rng.integers(0, n, q).astype(np.int32)
    pv = rng.integers(0, n, q).astype(np.int32)
    edge = np.isin(pu.astype(np.int64) * n + pv, keys)
    prec = lp.precision_at_k(ctx.score_pairs(pu, pv, "Z", "Y"), edge, [10, 100, 1000, 10000])
    _say(f"  dynamic AUC {auc_d:.4f} AP {ap_d:.4f}; static AUC {auc_s:.4f} AP {ap_s:.4f}; "
         f"precision@K {prec} ({int(edge.sum())} edges among {q} sampled pairs)")
    assert auc_d > 0.9 and ap_d > 0.9
    assert abs(auc_d - auc_s) <= 0.02 and abs(ap_d - ap_s) <= 0.02
    ctx.close()
