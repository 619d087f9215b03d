"""GPU flush and FP64 re-orthogonalisation against the oracle (Sec. 4.1).

Tolerances: a flush changes queries only by FP32 rounding of the rotated bases
(1e-5 of the largest entry); after re-orthogonalisation U^T U and V^T V are
within 1e-5 of I, singular values within 1e-5 * sigma_1 of the oracle's
re-orthogonalisation of the same exported state, and the product within 1e-5
relative Frobenius error; the PPR push invariant is kept to 2e-5.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.model import DAMFOracle
from oracle.reorth import reorthogonalize
from tests._checks import orth_err, product_rel_err, unit_factor
from workloads import c1_workload, chung_lu_directed

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


def _invariant_err(ctx, alpha, n):
    st = ctx.export_state()
    ip, ix = ctx.export_csr()
    A = sp.csr_matrix((np.ones(len(ix)), ix, ip), shape=(n, n))
    deg = np.asarray(A.sum(axis=1)).ravel()
    Pm = sp.diags(np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0.0)) @ A
    lhs = st["Ub"] - st["R"]
    rhs = (st["Zb"] - (1 - alpha) * (Pm @ st["Zb"])) / alpha
    return np.abs(lhs - rhs).max() / max(1.0, np.abs(st["Ub"]).max())


def _stream(rng, n, batches, k):
    for _ in range(batches):
        s, t = rng.integers(0, n, k), rng.integers(0, n, k)
        yield s, t, rng.choice(np.array([-1, 1, 1], dtype=np.int8), k)


def _ppr_ctx(P, n, m, d, seed, alpha=0.15, U=None, s=None, V=None):
    """Context on a Chung-Lu graph from the exact t-SVD, or from the given factors."""
    s0, t0 = chung_lu_directed(n, m, 2.1, seed)
    if U is None:
        orc = DAMFOracle(n, d, True, alpha=alpha, eps=1e-6, r=8, r_max=16, tau=1e-6)
        orc.init_exact(s0, t0)
        U, s, V = orc.U, orc.s, orc.V
    cfg = P.default_config(n, d, directed=True, alpha=alpha, eps=1e-6, max_core_rank=8,
                           max_side=16, tau=1e-6)
    return P.Context.init_factors(cfg, s0, t0, U, s, V)


def test_flush_keeps_queries_and_invariant(damf):
    _say("case flush")
    n, d, alpha = 500, 8, 0.15
    ctx = _ppr_ctx(damf, n, 4000, d, seed=31, alpha=alpha)
    for s, t, op in _stream(np.random.default_rng(6), n, 10, 30):
        ctx.update(s, t, op)
    before = ctx.export_state()
    assert np.abs(before["PU"] - np.eye(d)).max() > 1e-3  # the lazy projection is in use
    q = {w: ctx.query(w).astype(np.float64) for w in "XYZ"}
    ctx.flush()
    after = ctx.export_state()
    assert np.array_equal(after["PU"], np.eye(d)) and np.array_equal(after["PV"], np.eye(d))
    for key, pk in (("Ub", "PU"), ("Vb", "PV"), ("Zb", "PU"), ("R", "PU")):
        ref = before[key] @ before[pk]
        err = np.abs(after[key] - ref).max()
        _say(f"  {key}: |M_b P - flushed| {err:.2e} (max {np.abs(ref).max():.2e})")
        assert err <= 1e-5 * max(np.abs(ref).max(), 1e-30)
    for w in "XYZ":
        e = np.abs(ctx.query(w) - q[w]).max()
        assert e <= 1e-5 * np.abs(q[w]).max(), (w, e)
    inv = _invariant_err(ctx, alpha, n)
    _say(f"  invariant after flush {inv:.2e}")
    assert inv <= 2e-5
    ctx.close()


def _drifted_factors(n, d, seed, drift):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    V, _ = np.linalg.qr(rng.standard_normal((n, d)))
    U = U @ (np.eye(d) + drift * rng.standard_normal((d, d)))
    V = V @ (np.eye(d) + drift * rng.standard_normal((d, d)))
    s = np.sort(rng.uniform(2.0, 30.0, d))[::-1].copy()
    return U, s, V


@pytest.mark.parametrize("n,d", [(700, 8), (3000, 64), (2500, 128)])
def test_reorth_parity_with_oracle(damf, n, d):
    """Drifted factors, a few batches (P != I), then re-orthogonalise: compare with the
    oracle's re-orthogonalisation of the exported state U_b P_U, Sigma, V_b P_V."""
    _say(f"case reorth_parity n={n} d={d}")
    U, s, V = _drifted_factors(n, d, 7 + d, 1e-3)
    ctx = _ppr_ctx(damf, n, 8 * n, d, seed=33, U=U, s=s, V=V)
    for b, (s_, t_, op) in enumerate(_stream(np.random.default_rng(d), n, 3, 40)):
        ctx.update(s_, t_, op)
    st = ctx.export_state()
    Ue, Ve = st["Ub"] @ st["PU"], st["Vb"] @ st["PV"]
    se = ctx.singular_values()
    Uo, so, Vo = reorthogonalize(Ue, se, Ve)
    e0 = max(orth_err(Ue), orth_err(Ve))
    ctx.reorthogonalize()
    st2 = ctx.export_state()
    assert np.array_equal(st2["PU"], np.eye(d)) and np.array_equal(st2["PV"], np.eye(d))
    sg = ctx.singular_values()
    Ug, Vg = st2["Ub"], st2["Vb"]
    err_s = np.max(np.abs(sg - so)) / so[0]
    err_p = product_rel_err(Ug * sg, Vg, Uo * so, Vo)
    e1 = max(orth_err(Ug), orth_err(Vg))
    # singular vectors: gap-scaled agreement with the oracle's (sign aligned)
    gap = np.minimum(np.abs(np.diff(np.r_[np.inf, so])), np.abs(np.diff(np.r_[so, -np.inf]))) / so[0]
    sign = np.sign(np.sum(Ug * Uo, axis=0))
    dv = np.linalg.norm(Ug * sign - Uo, axis=0) * gap
    inv = _invariant_err(ctx, 0.15, n)
    _say(f"  orth {e0:.2e} -> {e1:.2e}, sigma err {err_s:.2e}, product err {err_p:.2e}, "
         f"gap-scaled vector err {dv.max():.2e}, invariant {inv:.2e}")
    assert e0 > 1e-4
    assert e1 <= 1e-5 and err_s <= 1e-5 and err_p <= 1e-5 and dv.max() <= 1e-5
    assert inv <= 2e-5
    ctx.enhance()
    assert ctx.residual_max() <= 1e-6
    ctx.close()


def test_reorth_every_keeps_c1_parity(damf):
    """C1 with a re-orthogonalisation every 16 batches: same factorisation as the oracle."""
    _say("case reorth_every_c1")
    w = c1_workload()
    orc = DAMFOracle(w["n"], w["d"], False, alpha=1.0, r=32, r_max=64, tau=1e-6).init_exact(*w["init"])
    cfg = damf.default_config(orc.n, orc.d, directed=False, alpha=1.0, max_core_rank=32,
                              max_side=64, tau=1e-6, reorth_every=16)
    ctx = damf.Context.init_factors(cfg, *w["init"], orc.U, orc.s, orc.V)
    n_re = 0
    for b, (s, t, op) in enumerate(w["stream"][:80]):
        orc.update(s, t, op)
        info = ctx.update(s, t, op)
        n_re += info["ms_reorth"] > 0
    sg = ctx.singular_values()
    X, Y = ctx.query("X"), ctx.query("Y")
    err_s = np.max(np.abs(sg - orc.s)) / orc.s[0]
    err_p = product_rel_err(X, Y, orc.X(), orc.Y())
    eo = max(orth_err(unit_factor(X, sg)), orth_err(unit_factor(Y, sg)))
    _say(f"  reorths {n_re}: sigma err {err_s:.2e} product err {err_p:.2e} orth {eo:.2e}")
    assert n_re == 5
    assert err_s <= 1e-5 and err_p <= 1e-5 and eo <= 1e-5
    ctx.close()


def test_reorth_every_keeps_residual_bound(damf):
    """A re-orthogonalisation rotates every row of R, so the push after it starts
    from every node: max |R| <= eps after each batch, with one due every 2 batches."""
    _say("case reorth_residual")
    n, eps = 800, 1e-5
    s0, t0 = chung_lu_directed(n, 8000, 2.1, 52)
    cfg = damf.default_config(n, 16, directed=True, alpha=0.15, eps=eps, oversample=10,
                              power_iters=2, seed=5, max_core_rank=8, max_side=16,
                              reorth_every=2)
    ctx = damf.Context.init(cfg, s0, t0)
    rng = np.random.default_rng(8)
    for b in range(6):
        k = 40
        s, t = rng.integers(0, n, k), rng.integers(0, n, k)
        op = rng.choice(np.array([-1, 1, 1], dtype=np.int8), k)
        info = ctx.update(s, t, op)
        rmax = ctx.residual_max()
        _say(f"  batch {b}: reorth {info['ms_reorth'] > 0} pushes {info['pushes']} max|R| {rmax:.2e}")
        assert rmax <= eps
    ctx.flush()
    ctx.query("Z", np.arange(10, dtype=np.int32))  # runs the push the flush left pending
    assert ctx.residual_max() <= eps
    ctx.close()


def test_reorth_rank_deficient_exact(damf):
    """d >= n: zero singular values get completed basis columns; X Y^T stays A."""
    _say("case reorth_rank_deficient")
    rng = np.random.default_rng(12)
    n = 24
    s0, t0 = rng.integers(0, n, 70), rng.integers(0, n, 70)
    orc = DAMFOracle(n, n, True, alpha=1.0, r=4, r_max=8, tau=1e-6).init_exact(s0, t0)
    cfg = damf.default_config(n, n, directed=True, alpha=1.0, max_core_rank=4, max_side=8, tau=1e-6)
    ctx = damf.Context.init_factors(cfg, s0, t0, orc.U, orc.s, orc.V)
    for s, t, op in _stream(rng, n, 6, 6):
        orc.update(s, t, op)
        ctx.update(s, t, op)
    ctx.reorthogonalize()
    st = ctx.export_state()
    A = orc.graph.dense()
    X, Y = ctx.query("X").astype(np.float64), ctx.query("Y").astype(np.float64)
    e_a = np.abs(X @ Y.T - A).max()
    e_o = max(orth_err(st["Ub"]), orth_err(st["Vb"]))
    _say(f"  |XY^T - A| {e_a:.2e} orth {e_o:.2e} zero sigmas {(ctx.singular_values() == 0).sum()}")
    assert e_a <= 1e-4 and e_o <= 1e-5
    ctx.close()


def test_reorth_refuses_a_basis_far_from_orthonormal(damf):
    _say("case reorth_refuses")
    rng = np.random.default_rng(13)
    n, d = 60, 4
    s0, t0 = rng.integers(0, n, 200), rng.integers(0, n, 200)
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    V, _ = np.linalg.qr(rng.standard_normal((n, d)))
    U[:, 1] = U[:, 0]  # rank-deficient U
    cfg = damf.default_config(n, d, directed=True, alpha=1.0, max_core_rank=4, max_side=8)
    ctx = damf.Context.init_factors(cfg, s0, t0, U, np.array([4.0, 3.0, 2.0, 1.0]), V)
    before = ctx.export_state()
    with pytest.raises(damf.DamfError) as ei:
        ctx.reorthogonalize()
    assert ei.value.status == 5
    after = ctx.export_state()
    for key in ("Ub", "Vb", "PU", "PV"):
        assert np.array_equal(before[key], after[key])
    ctx.flush()  # the context stays usable
    ctx.close()
