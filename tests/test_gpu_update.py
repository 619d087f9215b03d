"""GPU parity of the update path (Steps 1-3) and the graph store against the FP64 oracle.

Tolerances (stated here, derived in the design notes): singular values within
1e-5 * sigma_1; embedding product X Y^T within 1e-5 relative Frobenius error;
canonical CSR of A and A^T bit-exact; U = X Sigma^(-1/2) orthonormal to 1e-5.
"""
import sys

import numpy as np
import pytest

from oracle.graph import EdgeSet
from oracle.model import DAMFOracle
from tests._checks import orth_err, product_rel_err, unit_factor
from workloads import c1_workload, er_undirected

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


def _ctx_from_oracle(P, orc, init, **kw):
    cfg = P.default_config(orc.n, orc.d, directed=orc.directed, alpha=1.0,
                           max_core_rank=orc.r, max_side=orc.r_max, tau=orc.tau, **kw)
    return P.Context.init_factors(cfg, init[0], init[1], orc.U, orc.s, orc.V)


def _assert_csr(ctx, orc):
    for t in (False, True):
        ip, ix = ctx.export_csr(transpose=t)
        rp, rx = orc.graph.csr(transpose=t)
        assert np.array_equal(ip, rp), f"indptr transpose={t}"
        assert np.array_equal(ix, rx), f"indices transpose={t}"


@pytest.mark.parametrize("directed", [True, False])
def test_csr_edits_bit_exact(damf, directed):
    _say(f"case csr_edits directed={directed}")
    rng = np.random.default_rng(3)
    n, d = 50, 6
    s0, t0 = rng.integers(0, n, 200), rng.integers(0, n, 200)
    orc = DAMFOracle(n, d, directed, alpha=1.0, r=4, r_max=8, tau=1e-6).init_exact(s0, t0)
    ctx = _ctx_from_oracle(damf, orc, (s0, t0))
    _assert_csr(ctx, orc)
    for b in range(12):
        k = int(rng.integers(1, 40))
        s, t = rng.integers(0, n, k), rng.integers(0, n, k)
        op = rng.choice(np.array([-1, 1], dtype=np.int8), k)
        info_o = orc.update(s, t, op)
        info = ctx.update(s, t, op)
        assert info["net_entries"] == len(info_o["net"])
        assert info["chunks"] == len(info_o["chunks"])
        _assert_csr(ctx, orc)
    sg = ctx.singular_values()
    assert np.max(np.abs(sg - orc.s)) <= 1e-5 * orc.s[0]
    ctx.close()


def test_small_update_parity(damf):
    _say("case small_update_parity")
    rng = np.random.default_rng(5)
    n, d = 80, 8
    s0, t0 = rng.integers(0, n, 400), rng.integers(0, n, 400)
    orc = DAMFOracle(n, d, True, alpha=1.0, r=4, r_max=8, tau=1e-6).init_exact(s0, t0)
    ctx = _ctx_from_oracle(damf, orc, (s0, t0))
    for b in range(10):
        k = 12
        s, t = rng.integers(0, n, k), rng.integers(0, n, k)
        op = rng.choice(np.array([-1, 1], dtype=np.int8), k)
        orc.update(s, t, op)
        ctx.update(s, t, op)
        sg = ctx.singular_values()
        X, Y = ctx.query("X"), ctx.query("Y")
        err_s = np.max(np.abs(sg - orc.s)) / orc.s[0]
        err_p = product_rel_err(X, Y, orc.X(), orc.Y())
        _say(f"  batch {b}: sigma err {err_s:.2e} product err {err_p:.2e}")
        assert err_s <= 1e-5 and err_p <= 1e-5
    ctx.close()


@pytest.mark.parametrize("shared", [True, False])
def test_chunk_order_across_streams(damf, shared):
    """Step 3's solve-and-scatter of a chunk runs on a second stream beside the
    next chunk.  shared: every chunk of a batch has the same source row, so each
    front must wait for the previous scatter; else consecutive chunks touch
    disjoint rows and overlap.  Both must match the oracle chunk for chunk."""
    _say(f"case chunk_order shared={shared}")
    rng = np.random.default_rng(9)
    n, d, k = 200, 8, 40
    s0, t0 = rng.integers(0, n, 1500), rng.integers(0, n, 1500)
    orc = DAMFOracle(n, d, True, alpha=1.0, r=4, r_max=4, tau=1e-6).init_exact(s0, t0)
    ctx = _ctx_from_oracle(damf, orc, (s0, t0))
    for b in range(6):
        if shared:
            s = np.full(k, b, dtype=np.int64)
            t = rng.choice(n, k, replace=False)
        else:
            nodes = rng.permutation(n)[: 2 * k]
            s, t = nodes[:k], nodes[k:]
        op = np.ones(k, dtype=np.int8)
        orc.update(s, t, op)
        info = ctx.update(s, t, op)
        sg = ctx.singular_values()
        X, Y = ctx.query("X"), ctx.query("Y")
        err_s = np.max(np.abs(sg - orc.s)) / orc.s[0]
        err_p = product_rel_err(X, Y, orc.X(), orc.Y())
        _say(f"  batch {b}: chunks {info['chunks']} sigma err {err_s:.2e} product err {err_p:.2e}")
        assert info["chunks"] >= 8
        assert err_s <= 1e-5 and err_p <= 1e-5
    _assert_csr(ctx, orc)
    ctx.close()


def test_c1_parity(damf):
    """C1: undirected G(2000, 20000), d = 32, exact init on 90%, 200 batches of 10 inserts."""
    _say("case c1_parity")
    w = c1_workload()
    orc = DAMFOracle(w["n"], w["d"], False, alpha=1.0, r=32, r_max=64, tau=1e-6).init_exact(*w["init"])
    ctx = _ctx_from_oracle(damf, orc, w["init"])
    for b, (s, t, op) in enumerate(w["stream"]):
        orc.update(s, t, op)
        ctx.update(s, t, op)
        if b % 50 == 49:
            sg = ctx.singular_values()
            X, Y = ctx.query("X"), ctx.query("Y")
            err_s = np.max(np.abs(sg - orc.s)) / orc.s[0]
            err_p = product_rel_err(X, Y, orc.X(), orc.Y())
            eo = max(orth_err(unit_factor(X, sg)), orth_err(unit_factor(Y, sg)))
            _say(f"  batch {b}: sigma err {err_s:.2e} product err {err_p:.2e} orth {eo:.2e}")
            assert err_s <= 1e-5 and err_p <= 1e-5 and eo <= 1e-5
    _assert_csr(ctx, orc)
    ctx.close()


def test_exact_when_d_at_least_n(damf):
    _say("case exact_d_ge_n")
    rng = np.random.default_rng(11)
    n = 24
    s0, t0 = rng.integers(0, n, 80), rng.integers(0, n, 80)
    orc = DAMFOracle(n, n, True, alpha=1.0, r=4, r_max=8, tau=1e-6).init_exact(s0, t0)
    ctx = _ctx_from_oracle(damf, orc, (s0, t0))
    for _ in range(8):
        k = 6
        s, t = rng.integers(0, n, k), rng.integers(0, n, k)
        op = rng.choice(np.array([-1, 1], dtype=np.int8), k)
        orc.update(s, t, op)
        ctx.update(s, t, op)
        X, Y = ctx.query("X"), ctx.query("Y")
        A = orc.graph.dense()
        assert np.abs(X.astype(np.float64) @ Y.astype(np.float64).T - A).max() <= 1e-4
    ctx.close()


def test_invalid_ops_leave_state_unchanged(damf):
    _say("case invalid_ops")
    rng = np.random.default_rng(2)
    n, d = 40, 4
    s0, t0 = rng.integers(0, n, 120), rng.integers(0, n, 120)
    orc = DAMFOracle(n, d, True, alpha=1.0, r=4, r_max=8).init_exact(s0, t0)
    ctx = _ctx_from_oracle(damf, orc, (s0, t0))
    before = ctx.export_state()
    csr_before = ctx.export_csr()
    for bad in ([0, n], [-1, 3]):
        with pytest.raises(damf.DamfError) as ei:
            ctx.update(np.array(bad, dtype=np.int32), np.array([1, 2], dtype=np.int32),
                       np.array([1, 1], dtype=np.int8))
        assert ei.value.status == 2
    with pytest.raises(damf.DamfError):
        ctx.update(np.array([1], dtype=np.int32), np.array([2], dtype=np.int32),
                   np.array([3], dtype=np.int8))
    after = ctx.export_state()
    for key in ("Ub", "Vb", "PU", "PV"):
        assert np.array_equal(before[key], after[key])
    csr_after = ctx.export_csr()
    assert all(np.array_equal(a, b) for a, b in zip(csr_before, csr_after))
    # empty batch is a no-op
    info = ctx.update(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int8))
    assert info["chunks"] == 0
    ctx.close()


@pytest.mark.parametrize("d,r", [(64, 32), (128, 32), (128, 64)])
def test_wide_core_parity(damf, d, r):
    """d + r up to 192: the core SVD runs at padded sizes 128 and 192."""
    _say(f"case wide_core d={d} r={r}")
    from workloads import chung_lu_directed
    n, m = 1200, 16000
    s0, t0 = chung_lu_directed(n, m, 2.1, 41)
    orc = DAMFOracle(n, d, True, alpha=1.0, r=r, r_max=64, tau=1e-6).init_exact(s0, t0)
    ctx = _ctx_from_oracle(damf, orc, (s0, t0))
    rng = np.random.default_rng(d + r)
    for b in range(4):
        k = 150
        s, t = rng.integers(0, n, k), rng.integers(0, n, k)
        op = rng.choice(np.array([-1, 1, 1, 1], dtype=np.int8), k)
        io = orc.update(s, t, op)
        info = ctx.update(s, t, op)
        assert info["chunks"] == len(io["chunks"])
        sg = ctx.singular_values()
        X, Y = ctx.query("X"), ctx.query("Y")
        err_s = np.max(np.abs(sg - orc.s)) / orc.s[0]
        err_p = product_rel_err(X, Y, orc.X(), orc.Y())
        _say(f"  batch {b}: chunks {info['chunks']} max core {info['max_core']} sweeps "
             f"{info['sweeps']} sigma err {err_s:.2e} product err {err_p:.2e}")
        assert err_s <= 1e-5 and err_p <= 1e-5
    _assert_csr(ctx, orc)
    ctx.close()


def test_csr_build_hub_rows_beyond_lds(damf):
    """Rows longer than the LDS sort (32768 entries) take the global sorting network."""
    _say("case csr_hub_rows")
    rng = np.random.default_rng(8)
    n = 50000
    hub_out = rng.integers(0, n, 80000)           # node 7 -> ~40k distinct targets, duplicates
    hub_in = rng.integers(0, n, 70000)            # ~38k distinct sources -> node 11
    mid = rng.integers(0, n, 5000)                # a row between 2048 and 32768 entries
    s0 = np.concatenate([np.full(len(hub_out), 7), hub_in, np.full(len(mid), 3),
                         rng.integers(0, n, 20000)]).astype(np.int32)
    t0 = np.concatenate([hub_out, np.full(len(hub_in), 11), mid,
                         rng.integers(0, n, 20000)]).astype(np.int32)
    perm = rng.permutation(len(s0))
    s0, t0 = s0[perm], t0[perm]
    cfg = damf.default_config(n, 4, directed=True, alpha=1.0, max_core_rank=4, max_side=8,
                              oversample=4, power_iters=1)
    ctx = damf.Context.init(cfg, s0, t0)
    g = EdgeSet(n, True, s0, t0)
    for t in (False, True):
        ip, ix = ctx.export_csr(transpose=t)
        rp, rx = g.csr(transpose=t)
        assert np.array_equal(ip, rp) and np.array_equal(ix, rx), t
        assert np.diff(rp).max() > 32768, t
    ctx.close()


def test_csr_long_row_edits_in_place(damf):
    """Edits of rows longer than the LDS stage go through the global staging pool."""
    _say("case csr_long_row_edits")
    rng = np.random.default_rng(12)
    n = 30000
    s0 = np.concatenate([np.full(20000, 5), rng.integers(0, n, 15000),
                         rng.integers(0, n, 30000)]).astype(np.int32)
    t0 = np.concatenate([rng.permutation(n)[:20000], np.full(15000, 9),
                         rng.integers(0, n, 30000)]).astype(np.int32)
    cfg = damf.default_config(n, 4, directed=True, alpha=1.0, max_core_rank=8, max_side=16,
                              oversample=4, power_iters=1)
    ctx = damf.Context.init(cfg, s0, t0)
    g = EdgeSet(n, True, s0, t0)
    for b in range(6):
        k = 400
        s = np.where(rng.random(k) < 0.5, 5, rng.integers(0, n, k)).astype(np.int32)
        t = np.where(s == 5, rng.integers(0, n, k), np.where(rng.random(k) < 0.5, 9,
                                                            rng.integers(0, n, k))).astype(np.int32)
        op = rng.choice(np.array([-1, 1], dtype=np.int8), k)
        g.apply(s, t, op)
        ctx.update(s, t, op)
        for tr in (False, True):
            ip, ix = ctx.export_csr(transpose=tr)
            rp, rx = g.csr(transpose=tr)
            assert np.array_equal(ip, rp) and np.array_equal(ix, rx), (b, tr)
    ctx.close()


def test_csr_pool_compaction(damf):
    """Rows that keep outgrowing their reservation leak pool space until a compaction."""
    _say("case csr_pool_compaction")
    rng = np.random.default_rng(13)
    n = 4000
    s0, t0 = rng.integers(0, n, 2000).astype(np.int32), rng.integers(0, n, 2000).astype(np.int32)
    cfg = damf.default_config(n, 8, directed=True, alpha=1.0, max_core_rank=64, max_side=64,
                              oversample=4, power_iters=1)
    ctx = damf.Context.init(cfg, s0, t0)
    g = EdgeSet(n, True, s0, t0)
    for b in range(60):
        k = 8192
        s = rng.integers(0, n, k).astype(np.int32)
        t = rng.integers(0, n, k).astype(np.int32)
        op = np.ones(k, dtype=np.int8)
        g.apply(s, t, op)
        ctx.update(s, t, op)
        if b % 20 == 19 or b == 59:
            for tr in (False, True):
                ip, ix = ctx.export_csr(transpose=tr)
                rp, rx = g.csr(transpose=tr)
                assert np.array_equal(ip, rp) and np.array_equal(ix, rx), (b, tr)
            _say(f"  batch {b}: {len(ix)} edges")
    ctx.close()
