"""GPU parity of the randomized t-SVD initialisation (Appendix A, Algorithm 3).

Exact when rank(A) <= d + p (a block graph); otherwise compared with the
oracle's randomized t-SVD from the same SplitMix64 sketch.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.factor import tsvd_randomized
from oracle.graph import EdgeSet
from tests._checks import orth_err, product_rel_err, unit_factor
from workloads import block_graph, chung_lu_directed

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


@pytest.mark.parametrize("n", [300, 1000])
def test_rsvd_exact_on_low_rank(damf, n):
    _say(f"case rsvd_exact n={n}")
    s0, t0 = block_graph(n, 6, seed=3)
    d, p = 8, 4
    cfg = damf.default_config(n, d, directed=True, alpha=1.0, oversample=p, power_iters=2, seed=7)
    ctx = damf.Context.init(cfg, s0, t0)
    A = EdgeSet(n, True, s0, t0).dense()
    X, Y = ctx.query("X").astype(np.float64), ctx.query("Y").astype(np.float64)
    err = np.abs(X @ Y.T - A).max()
    sv = np.linalg.svd(A, compute_uv=False)[:d]
    sg = ctx.singular_values()
    fb = ctx.init_info()["qr_fallbacks"]
    _say(f"  max|XY^T - A| {err:.2e} sigma err {np.abs(sg - sv).max() / sv[0]:.2e} "
         f"QR fallbacks {fb}")
    # rank 6 < d + p = 12: every sketch's Gram is singular, so the QRs take
    # the Householder TSQR
    assert fb > 0
    assert err <= 1e-4
    assert np.abs(sg - sv).max() <= 1e-5 * sv[0]
    ctx.close()


def test_rsvd_matches_oracle_same_sketch(damf):
    _say("case rsvd_parity")
    n, m, d, p, q, seed = 3000, 30000, 16, 10, 2, 5
    s0, t0 = chung_lu_directed(n, m, 2.1, 31)
    A = sp.csr_matrix((np.ones(m), (s0, t0)), shape=(n, n))
    U, s, V = tsvd_randomized(A, d, p, q, seed)
    cfg = damf.default_config(n, d, directed=True, alpha=1.0, oversample=p, power_iters=q, seed=seed)
    ctx = damf.Context.init(cfg, s0, t0)
    sg = ctx.singular_values()
    X, Y = ctx.query("X"), ctx.query("Y")
    err_s = np.abs(sg - s).max() / s[0]
    err_p = product_rel_err(X, Y, U * np.sqrt(s), V * np.sqrt(s))
    eo = max(orth_err(unit_factor(X, sg)), orth_err(unit_factor(Y, sg)))
    fb = ctx.init_info()["qr_fallbacks"]
    _say(f"  sigma err {err_s:.2e} product err {err_p:.2e} orth {eo:.2e} QR fallbacks {fb}")
    assert fb == 0  # full-rank sketches: every QR ran as CholeskyQR2
    assert err_s <= 1e-5 and err_p <= 1e-5 and eo <= 1e-5
    ctx.close()


def _hub_graph(n, seed):
    """Sparse random graph plus hub rows and columns far longer than one SpMM segment."""
    rng = np.random.default_rng(seed)
    s = [rng.integers(0, n, 6 * n)]
    t = [rng.integers(0, n, 6 * n)]
    for h, deg in ((3, 9000), (17, 2500), (41, 700)):
        s += [np.full(deg, h), rng.integers(0, n, deg)]
        t += [rng.integers(0, n, deg), np.full(deg, h + 1)]
    s, t = np.concatenate(s).astype(np.int32), np.concatenate(t).astype(np.int32)
    g = EdgeSet(n, True, s, t)
    ip, ix = g.csr()
    src = np.repeat(np.arange(n), np.diff(ip)).astype(np.int32)
    return src, ix.astype(np.int32)


def test_rsvd_parity_with_hub_rows(damf):
    """Rows split into SpMM segments (out- and in-CSR) give the oracle's randomized t-SVD."""
    _say("case rsvd_hub_rows")
    n, d, p, q, seed = 6000, 16, 10, 2, 9
    s0, t0 = _hub_graph(n, 4)
    A = sp.csr_matrix((np.ones(len(s0)), (s0, t0)), shape=(n, n))
    assert np.diff(A.indptr).max() > 2000 and np.diff(A.tocsc().indptr).max() > 2000
    U, s, V = tsvd_randomized(A, d, p, q, seed)
    cfg = damf.default_config(n, d, directed=True, alpha=1.0, oversample=p, power_iters=q, seed=seed)
    ctx = damf.Context.init(cfg, s0, t0)
    sg = ctx.singular_values()
    X, Y = ctx.query("X"), ctx.query("Y")
    err_s = np.abs(sg - s).max() / s[0]
    err_p = product_rel_err(X, Y, U * np.sqrt(s), V * np.sqrt(s))
    fb = ctx.init_info()["qr_fallbacks"]
    _say(f"  sigma err {err_s:.2e} product err {err_p:.2e} QR fallbacks {fb}")
    assert fb == 0
    assert err_s <= 1e-5 and err_p <= 1e-5
    ctx.close()


def test_ppr_init_with_hub_rows(damf):
    """Propagation rounds over split rows keep the push invariant X - R = (Z - (1-a) P Z) / a."""
    _say("case ppr_init_hub_rows")
    n, d, alpha = 6000, 8, 0.15
    s0, t0 = _hub_graph(n, 5)
    cfg = damf.default_config(n, d, directed=True, alpha=alpha, eps=1e-6, oversample=4, seed=2)
    ctx = damf.Context.init(cfg, s0, t0)
    st = ctx.export_state()
    A = sp.csr_matrix((np.ones(len(s0)), (s0, t0)), shape=(n, n))
    deg = np.asarray(A.sum(axis=1)).ravel()
    Pm = sp.diags(np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0.0)) @ A
    err = np.abs((st["Ub"] - st["R"]) - (st["Zb"] - (1 - alpha) * (Pm @ st["Zb"])) / alpha).max()
    _say(f"  invariant err {err:.2e} max|R| {ctx.residual_max():.2e}")
    assert err <= 2e-5 * max(1.0, np.abs(st["Ub"]).max())
    assert ctx.residual_max() <= 1e-6
    ctx.close()
