"""GPU parity of Step 4 (PPR enhancement) against the oracle's PPR series.

Bound used: Z_b within eps of PPR(U_b) entrywise (max |R| <= eps and Pi >= 0
with row sums <= 1), so after the query's P_U Sigma^(1/2) and the sign
alignment of singular vectors,
  |Z_gpu - Z_orc| <= max |X_gpu - X_orc| + eps * max_c (sum_k |P_U[k, c]|) sqrt(sigma_c).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.model import DAMFOracle
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


def _make(P, n, m, d, alpha, eps, seed, directed=True):
    s0, t0 = chung_lu_directed(n, m, 2.1, seed)
    orc = DAMFOracle(n, d, directed, alpha=alpha, eps=eps, r=8, r_max=16, tau=1e-6).init_exact(s0, t0)
    cfg = P.default_config(n, d, directed=directed, alpha=alpha, eps=eps, max_core_rank=8,
                           max_side=16, tau=1e-6)
    ctx = P.Context.init_factors(cfg, s0, t0, orc.U, orc.s, orc.V)
    return orc, ctx


def _check_z(ctx, orc, eps):
    sg = ctx.singular_values()
    X = ctx.query("X").astype(np.float64)
    Z = ctx.query("Z").astype(np.float64)
    Xo, Zo = orc.X(), orc.Z()
    sign = np.sign((X * Xo).sum(axis=0))
    sign[sign == 0] = 1.0
    dx = np.abs(X * sign - Xo).max()
    st = ctx.export_state()
    scale = (np.abs(st["PU"]).sum(axis=0) * np.sqrt(sg)).max()
    dz = np.abs(Z * sign - Zo).max()
    bound = dx + eps * scale + 1e-6 * np.abs(Zo).max()
    _say(f"  |dX| {dx:.2e} |dZ| {dz:.2e} bound {bound:.2e} max|R| {ctx.residual_max():.2e}")
    assert dz <= bound
    assert ctx.residual_max() <= eps


def test_ppr_initial_propagation(damf):
    _say("case ppr_init")
    orc, ctx = _make(damf, 400, 3000, 8, 0.15, 1e-6, seed=21)
    _check_z(ctx, orc, 1e-6)
    assert ctx.residual_max() <= 0.5e-6  # the start propagates to eps / 2
    ctx.close()


def test_ppr_dynamic_push(damf):
    _say("case ppr_dynamic")
    n = 400
    orc, ctx = _make(damf, n, 3000, 8, 0.15, 1e-6, seed=22)
    rng = np.random.default_rng(9)
    for b in range(8):
        k = 30
        s, t = rng.integers(0, n, k), rng.integers(0, n, k)
        op = rng.choice(np.array([-1, 1, 1], dtype=np.int8), k)
        orc.update(s, t, op)
        info = ctx.update(s, t, op)
        _say(f" batch {b}: rounds {info['push_rounds']} pushes {info['pushes']}")
    _check_z(ctx, orc, 1e-6)
    ctx.close()


def test_z_query_runs_pending_enhance(damf):
    """With auto_enhance = 0 the batches leave Step 4 pending; a Z query runs it first,
    so Z matches the oracle's PPR(X) as with auto_enhance = 1."""
    _say("case ppr_pending")
    n, eps = 400, 1e-6
    s0, t0 = chung_lu_directed(n, 3000, 2.1, 24)
    orc = DAMFOracle(n, 8, True, alpha=0.15, eps=eps, r=8, r_max=16, tau=1e-6).init_exact(s0, t0)
    cfg = damf.default_config(n, 8, directed=True, alpha=0.15, eps=eps, max_core_rank=8,
                              max_side=16, tau=1e-6, auto_enhance=0)
    ctx = damf.Context.init_factors(cfg, s0, t0, orc.U, orc.s, orc.V)
    rng = np.random.default_rng(10)
    for b in range(6):
        k = 30
        s, t = rng.integers(0, n, k), rng.integers(0, n, k)
        op = rng.choice(np.array([-1, 1, 1], dtype=np.int8), k)
        orc.update(s, t, op)
        info = ctx.update(s, t, op)
        assert info["push_rounds"] == 0
    assert ctx.residual_max() > eps  # Step 4 still pending
    _check_z(ctx, orc, eps)          # the Z query inside runs it
    ctx.close()


def test_ppr_invariant_property(damf):
    """X - R == (Z_b - (1 - alpha) P Z_b) / alpha on the GPU's own state (any size)."""
    _say("case ppr_invariant")
    n, alpha = 600, 0.15
    orc, ctx = _make(damf, n, 5000, 8, alpha, 1e-5, seed=23)
    rng = np.random.default_rng(4)
    for _ in range(5):
        k = 40
        s, t = rng.integers(0, n, k), rng.integers(0, n, k)
        op = rng.choice(np.array([-1, 1], dtype=np.int8), k)
        orc.update(s, t, op)
        ctx.update(s, t, op)
    st = ctx.export_state()
    ip, ix = ctx.export_csr()
    A = sp.csr_matrix((np.ones(len(ix)), ix, ip), shape=(n, n))
    deg = np.asarray(A.sum(axis=1)).ravel()
    inv = np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0.0)
    Pm = sp.diags(inv) @ A
    lhs = st["Ub"] - st["R"]
    rhs = (st["Zb"] - (1 - alpha) * (Pm @ st["Zb"])) / alpha
    err = np.abs(lhs - rhs).max()
    _say(f"  invariant err {err:.2e} (|U_b| max {np.abs(st['Ub']).max():.2e})")
    assert err <= 2e-5 * max(1.0, np.abs(st["Ub"]).max())
    ctx.close()


def test_alpha_one_gives_no_enhancement(damf):
    _say("case alpha_one")
    orc, ctx = _make(damf, 200, 1200, 6, 1.0, 1e-5, seed=24)
    assert np.array_equal(ctx.query("Z"), ctx.query("X"))
    ctx.close()
