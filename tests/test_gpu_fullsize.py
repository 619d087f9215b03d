"""The C2 workload at its full size (directed Chung-Lu 2.1, n = 1e6, m = 1e7,
d = 128, batches of 1,000 ops) in the configuration bench.py times (chunk rank
64, r_max 64), checked on outputs the oracle computes row by row and on
properties that hold at any size.

- Steps 1-3 against the FP64 oracle: both start from the same seeded
  orthonormal factors on the same graph and apply one batch; singular values
  and the embedding product X Y^T restricted to a row sample (every touched
  row plus 2,000 random rows) agree to the FP32 tolerance 1e-5.
- CSR edits bit-exact after two batches, against the edge set the
  definition gives (ops in order on a set: the last op on an edge decides),
  written out with numpy sorts at this size.
- Step 4: the PPR invariant U_b - R = (Z_b - (1 - alpha) P Z_b) / alpha on a
  row sample and max |R| <= eps, after the randomized init and two batches.
"""
import sys

import numpy as np
import pytest

from oracle.graph import EdgeSet
from oracle.model import DAMFOracle
from tests._checks import product_rel_err
from workloads import chung_lu_workload

pytestmark = pytest.mark.gpu

N, M, D, BATCH, SEED = 1_000_000, 10_000_000, 128, 1000, 2


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


@pytest.fixture(scope="module")
def c2():
    _say("case c2 workload")
    return chung_lu_workload(N, M, 2.1, SEED, 2, BATCH, 0.95, d=D)


def test_c2_steps_1_3_parity_sampled(damf, c2):
    _say("case c2_steps_1_3 (n=1e6, m=1e7, d=128, one batch of 1000)")
    rng = np.random.default_rng(12345)
    U, _ = np.linalg.qr(rng.standard_normal((N, D)))
    V, _ = np.linalg.qr(rng.standard_normal((N, D)))
    s = np.sort(rng.uniform(40.0, 260.0, D))[::-1].copy()
    orc = DAMFOracle(N, D, True, alpha=1.0, r=64, r_max=64, tau=1e-6)
    orc.graph = EdgeSet(N, True, *c2["init"])
    orc.U, orc.V, orc.s = U.copy(), V.copy(), s.copy()
    cfg = damf.default_config(N, D, directed=True, alpha=1.0, max_core_rank=64, max_side=64, tau=1e-6)
    ctx = damf.Context.init_factors(cfg, *c2["init"], U, s, V)
    src, dst, op = c2["stream"][0]
    orc.update(src, dst, op)
    info = ctx.update(src, dst, op)
    rows = np.unique(np.concatenate([src, dst, rng.choice(N, 2000, replace=False)])).astype(np.int32)
    Xg = ctx.query("X", rows).astype(np.float64)
    Yg = ctx.query("Y", rows).astype(np.float64)
    Xo, Yo = orc.X()[rows], orc.Y()[rows]
    sg = ctx.singular_values()
    err_s = np.max(np.abs(sg - orc.s)) / orc.s[0]
    err_p = product_rel_err(Xg, Yg, Xo, Yo)
    _say(f"  chunks {info['chunks']} sweeps {info['sweeps']} rows {len(rows)}: "
         f"sigma err {err_s:.2e} product err {err_p:.2e}")
    assert err_s <= 1e-5 and err_p <= 1e-5
    ctx.close()


def test_c2_csr_and_ppr_invariant(damf, c2):
    import scipy.sparse as sp
    import torch
    _say("case c2_csr_ppr (randomized init, alpha 0.15, eps 1e-5, two batches)")
    alpha, eps = 0.15, 1e-5
    cfg = damf.default_config(N, D, directed=True, alpha=alpha, eps=eps, oversample=10, power_iters=2,
                              seed=SEED, max_core_rank=64, max_side=64)
    src0 = torch.from_numpy(c2["init"][0]).cuda()
    dst0 = torch.from_numpy(c2["init"][1]).cuda()
    ctx = damf.Context.init(cfg, src0, dst0)
    ops = []
    for b in range(2):
        s, t, o = c2["stream"][b]
        ctx.update(s, t, o)
        ops.append((s, t, o))
    # the edge set after the ops: initial keys, then for every key touched the
    # last op decides presence
    key0 = c2["init"][0].astype(np.int64) * N + c2["init"][1].astype(np.int64)
    ks = np.concatenate([a.astype(np.int64) * N + b.astype(np.int64) for a, b, _ in ops])
    os_ = np.concatenate([o.astype(np.int8) for _, _, o in ops])
    last = len(ks) - 1 - np.unique(ks[::-1], return_index=True)[1]
    ins, dels = ks[last][os_[last] > 0], ks[last][os_[last] < 0]
    final = np.union1d(np.setdiff1d(key0, dels), ins)
    ip, ix = ctx.export_csr()
    exp_ip = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(final // N, minlength=N), out=exp_ip[1:])
    assert np.array_equal(ip, exp_ip)
    assert np.array_equal(ix, (final % N).astype(np.int32))
    _say(f"  CSR exact: {len(ix)} edges")
    # invariant on a row sample
    rmax = ctx.residual_max()
    st = ctx.export_state()
    rng = np.random.default_rng(7)
    rows = rng.choice(N, 4000, replace=False)
    A = sp.csr_matrix((np.ones(len(ix)), ix, ip), shape=(N, N))
    deg = np.diff(ip).astype(np.float64)
    sub = A[rows]
    pz = (sub @ st["Zb"]) / np.maximum(deg[rows], 1.0)[:, None]
    lhs = st["Ub"][rows] - st["R"][rows]
    rhs = (st["Zb"][rows] - (1 - alpha) * pz) / alpha
    err = np.abs(lhs - rhs).max()
    scale = max(1.0, np.abs(st["Ub"]).max())
    _say(f"  invariant err {err:.2e} (|U_b| max {scale:.2e}), max|R| {rmax:.2e}")
    assert rmax <= eps
    assert err <= 2e-5 * scale
    ctx.close()
