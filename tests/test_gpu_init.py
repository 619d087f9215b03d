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
    _say(f"  max|XY^T - A| {err:.2e} sigma err {np.abs(sg - sv).max() / sv[0]:.2e}")
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
    _say(f"  sigma err {err_s:.2e} product err {err_p:.2e} orth {eo:.2e}")
    assert err_s <= 1e-5 and err_p <= 1e-5 and eo <= 1e-5
    ctx.close()
