"""GPU parity on the paths the benchmark configurations run, against the FP64 oracle.

1. Randomized t-SVD (Appendix A, Algorithm 3) at the benchmark shape d = 128,
   p = 10 (l = 138: the nine-tile resident-B tall product and the 45-tile
   FP64-MFMA Gram of CholeskyQR2) and at p = 20 (l = 148: the strided
   twelve-tile product), on a Chung-Lu graph of n = 20,000 that spans many
   256-row blocks.  Same SplitMix64 sketch on both sides.
2. Step 4 push on nodes with more than 64 in-neighbours (the heavy-row push:
   70 up to 9,000 in-neighbours), after the initial propagation and after
   dynamic batches that change hub rows.
3. C1 as configured (undirected G(2000, 20000), d = 32, exact init on 90%,
   200 batches of 10 inserts, alpha = 0.15, eps = 1e-4), checked at batches
   50, 100, 150 and 200.

Bars (FP32 state against the FP64 oracle):
- singular values: max |s_gpu - s_orc| <= 1e-5 s_1;
- leading subspaces (Wedin): sin angle(U_gpu[:, :j], U_orc[:, :j]) <= 1e-5 / g_j
  for every j with relative gap g_j = (s_j - s_{j+1}) / s_1 > 0, same for V;
- embedding product X Y^T: relative Frobenius error <= 1e-5 / g_d, capped at
  1e-5 when g_d >= 1;
- rows of X Y^T: each sampled row's relative error <= 1e-4 / g_d (a row is a
  d-term combination of the columns, so it can carry up to about sqrt(d)
  times the Frobenius average; 1e-4 leaves that factor at d = 128);
- reconstruction error ||A - X Y^T||_F^2: within 1e-5 ||A||_F^2 of the
  oracle's (first-order insensitive to the basis);
- PPR (Sec. 4.4): the GPU's Z_b within eps + 1e-6 max|Z| of the PPR series of
  the GPU's own U_b (isolates Step 4 from SVD drift).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.factor import tsvd_randomized
from oracle.graph import EdgeSet
from oracle.model import DAMFOracle
from oracle.ppr import ppr_series
from tests._checks import (gap_scaled_ratio, orth_err, product_rel_err, recon_err2,
                           relative_gaps, row_product_errs, subspace_sines, unit_factor)
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


def _csr(ctx, n):
    ip, ix = ctx.export_csr()
    return sp.csr_matrix((np.ones(len(ix)), ix, ip), shape=(n, n))


def _factor_checks(tag, sg, X, Y, s_orc, s_full, U_orc, V_orc, A, rows):
    """The singular-value, subspace, product, row and reconstruction bars."""
    d = len(s_orc)
    gaps = relative_gaps(s_full, d)
    g_d = gaps[-1]
    Xo, Yo = U_orc * np.sqrt(s_orc), V_orc * np.sqrt(s_orc)
    err_s = np.abs(sg - s_orc).max() / s_orc[0]
    su = subspace_sines(unit_factor(X, sg), U_orc)
    sv = subspace_sines(unit_factor(Y, sg), V_orc)
    ru, rv = gap_scaled_ratio(su, gaps), gap_scaled_ratio(sv, gaps)
    err_p = product_rel_err(X, Y, Xo, Yo)
    bar_p = 1e-5 / min(1.0, g_d)
    rowe = row_product_errs(X, Y, Xo, Yo, rows)
    bar_r = 1e-4 / min(1.0, g_d)
    nnz = float(A.nnz)
    drec = abs(recon_err2(A, X, Y) - recon_err2(A, Xo, Yo)) / nnz
    eo = max(orth_err(unit_factor(X, sg)), orth_err(unit_factor(Y, sg)))
    _say(f"  {tag}: sigma {err_s:.2e}  sin-ratio U {ru:.2e} V {rv:.2e} (sin_d {su[-1]:.2e}, "
         f"g_d {g_d:.2e})  product {err_p:.2e} (bar {bar_p:.1e})  rows max {rowe.max():.2e} "
         f"median {np.median(rowe):.2e} ({len(rowe)} rows)  recon {drec:.2e}  orth {eo:.2e}")
    assert err_s <= 1e-5
    assert ru <= 1.0 and rv <= 1.0
    assert err_p <= bar_p
    assert rowe.max() <= bar_r
    assert drec <= 1e-5
    assert eo <= 1e-5


@pytest.mark.parametrize("p", [10, 20])
def test_rsvd_benchmark_shape(damf, p):
    n, m, d, q, seed = 20_000, 200_000, 128, 2, 11
    _say(f"case rsvd d={d} p={p} (l={d + p}) n={n} m={m}")
    s0, t0 = chung_lu_directed(n, m, 2.1, 51)
    A = sp.csr_matrix((np.ones(m), (s0, t0)), shape=(n, n))
    U, s, V, s_full = tsvd_randomized(A, d, p, q, seed, full_spectrum=True)
    cfg = damf.default_config(n, d, directed=True, alpha=1.0, oversample=p, power_iters=q,
                              seed=seed)
    ctx = damf.Context.init(cfg, s0, t0)
    fb = ctx.init_info()["qr_fallbacks"]
    _say(f"  QR fallbacks {fb}")
    assert fb == 0  # every tall QR ran as CholeskyQR2 (Gram on FP64 MFMA + MFMA product)
    sg = ctx.singular_values()
    X, Y = ctx.query("X"), ctx.query("Y")
    rows = np.random.default_rng(1).choice(n, 4000, replace=False)
    _factor_checks(f"l={d + p}", sg, X, Y, s, s_full, U, V, A, rows)
    ctx.close()


def _hub_stream_graph(n, seed):
    """Random directed graph (5 n edges) plus nodes with 70 .. 9,000 in-neighbours,
    each also with out-edges, so batches can change their rows."""
    rng = np.random.default_rng(seed)
    hubs = np.array([11, 222, 3333, 4444, 5555], dtype=np.int64)
    indeg = [70, 300, 1500, 3000, 9000]
    s = [rng.integers(0, n, 5 * n)]
    t = [rng.integers(0, n, 5 * n)]
    for h, k in zip(hubs, indeg):
        s += [rng.choice(n, k, replace=False), np.full(40, h)]
        t += [np.full(k, h), rng.integers(0, n, 40)]
    g = EdgeSet(n, True, np.concatenate(s), np.concatenate(t))
    ip, ix = g.csr()
    src = np.repeat(np.arange(n), np.diff(ip)).astype(np.int32)
    return src, ix.astype(np.int32), hubs


def _check_ppr(ctx, A, alpha, eps, tag):
    st = ctx.export_state()
    Zs = ppr_series(A, st["Ub"], alpha)
    err = np.abs(st["Zb"] - Zs).max()
    bar = eps + 1e-6 * np.abs(Zs).max()
    _say(f"  {tag}: |Z_b - PPR(U_b)| {err:.2e} bar {bar:.2e} max|R| {ctx.residual_max():.2e}")
    assert err <= bar
    assert ctx.residual_max() <= eps
    return st, Zs


def test_push_heavy_rows_vs_series(damf):
    n, d, alpha, eps = 20_000, 8, 0.15, 1e-6
    _say(f"case heavy-row push n={n} d={d} eps={eps}")
    s0, t0, hubs = _hub_stream_graph(n, 61)
    A0 = sp.csr_matrix((np.ones(len(s0)), (s0, t0)), shape=(n, n))
    assert np.diff(A0.tocsc().indptr).max() >= 8990  # one hub: 9,000 in-neighbours (less a self-loop)
    cfg = damf.default_config(n, d, directed=True, alpha=alpha, eps=eps, oversample=6, seed=3,
                              max_core_rank=16, max_side=32)
    ctx = damf.Context.init(cfg, s0, t0)
    _check_ppr(ctx, _csr(ctx, n), alpha, eps, "after init propagation")
    rng = np.random.default_rng(62)
    heavy_edges = 0
    for b in range(6):
        k = 120
        # out-edges of hubs change (structural fix-up of hub rows, so hubs enter
        # the frontier), new in-edges of hubs, and random edits
        hs = rng.choice(hubs, 40)
        s = np.concatenate([hs, rng.integers(0, n, 40), rng.integers(0, n, 40)])
        t = np.concatenate([rng.integers(0, n, 40), rng.choice(hubs, 40), rng.integers(0, n, 40)])
        op = rng.choice(np.array([-1, 1, 1], dtype=np.int8), k)
        info = ctx.update(s.astype(np.int32), t.astype(np.int32), op)
        heavy_edges = max(heavy_edges, info["push_edges"])
        _say(f"  batch {b}: rounds {info['push_rounds']} pushes {info['pushes']} "
             f"edges {info['push_edges']}")
        if b % 2 == 1:
            _check_ppr(ctx, _csr(ctx, n), alpha, eps, f"after batch {b}")
    # a pushed hub traverses all of its in-neighbours
    assert heavy_edges >= 9000
    ctx.close()


def test_c1_as_configured(damf):
    """C1 end to end with Step 4 on (alpha = 0.15, eps = 1e-4)."""
    _say("case c1 configured alpha=0.15 eps=1e-4")
    w = c1_workload()
    n, d, alpha, eps = w["n"], w["d"], 0.15, 1e-4
    orc = DAMFOracle(n, d, False, alpha=alpha, eps=eps, r=32, r_max=64,
                     tau=1e-6).init_exact(*w["init"])
    cfg = damf.default_config(n, d, directed=False, alpha=alpha, eps=eps, max_core_rank=32,
                              max_side=64, tau=1e-6)
    ctx = damf.Context.init_factors(cfg, w["init"][0], w["init"][1], orc.U, orc.s, orc.V)
    for b, (s, t, op) in enumerate(w["stream"]):
        orc.update(s, t, op)
        ctx.update(s, t, op)
        if b % 50 == 49:
            A = orc.graph.scipy()
            s_full = np.linalg.svd(A.toarray(), compute_uv=False)[: d + 1]
            sg = ctx.singular_values()
            X, Y = ctx.query("X"), ctx.query("Y")
            _factor_checks(f"batch {b + 1}", sg, X, Y, orc.s, s_full, orc.U, orc.V, A,
                           np.arange(n))
            st, Zs = _check_ppr(ctx, _csr(ctx, n), alpha, eps, f"batch {b + 1}")
            # the queried Z = Z_b P_U Sigma^(1/2) against PPR(U_b) P_U Sigma^(1/2)
            Zq = ctx.query("Z").astype(np.float64)
            Zref = (Zs @ st["PU"]) * np.sqrt(sg)[None, :]
            scale = (np.abs(st["PU"]).sum(axis=0) * np.sqrt(sg)).max()
            dz = np.abs(Zq - Zref).max()
            _say(f"  batch {b + 1}: |Z - PPR(X)| {dz:.2e} bar {eps * scale:.2e}")
            assert dz <= eps * scale + 1e-6 * np.abs(Zref).max()
    ip, ix = ctx.export_csr()
    rp, rx = orc.graph.csr()
    assert np.array_equal(ip, rp) and np.array_equal(ix, rx)
    ctx.close()
