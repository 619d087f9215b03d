"""Node counts past what one dispatch can address element by element.

At n = 34,600,000 and d = 128 an n x d basis has 4.4e9 entries and a launch
with one workgroup of 256 per node would need 8.9e9 work-items; a dispatch
holds fewer than 2^32, so every elementwise and per-node kernel (CSR build,
sketch, BF16-pair encode/decode, PPR start) has to stride over its range.

The graph is a disjoint union of 120 directed bicliques R_i -> C_i with
|R_i| = a_i, |C_i| = b_i, their nodes scattered over the whole id range.  A
then has rank 120 <= d and a closed-form t-SVD: sigma_i = sqrt(a_i b_i),
u_i = 1_{R_i} / sqrt(a_i), v_i = 1_{C_i} / sqrt(b_i) (Section 4.1's rank-d
factorisation is exact), and the randomized init (Appendix A, Algorithm 3)
recovers it to FP32 rounding because the sketch of width d + p spans the
range of A.  Checked, for the FP32 form and the precision form:
- the CSR export equals the edge set (bit-exact);
- the singular values equal the closed form, the rest are zero;
- X Y^T equals A on a row sample that holds every biclique node and the
  highest node ids (isolated nodes must give zero rows);
- max |R| <= eps after the PPR start and after one batch of 100 inserts
  among biclique nodes, and the CSR after that batch equals the edge set
  with the inserts.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N, D, BLOCKS = 34_600_000, 128, 120


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


def _bicliques(seed):
    rng = np.random.default_rng(seed)
    a = 3 + np.arange(BLOCKS) % 5
    b = 4 + np.arange(BLOCKS)
    ids = rng.choice(N, int(a.sum() + b.sum()), replace=False).astype(np.int32)
    # some blocks entirely among the highest ids, past 2^32 / d
    top = np.arange(N - int(a[:10].sum() + b[:10].sum()), N, dtype=np.int32)
    ids = np.concatenate([top, ids[~np.isin(ids, top)]])
    rows, cols, src, dst, pos = [], [], [], [], 0
    for i in range(BLOCKS):
        r = ids[pos:pos + a[i]]
        pos += a[i]
        c = ids[pos:pos + b[i]]
        pos += b[i]
        rows.append(r)
        cols.append(c)
        src.append(np.repeat(r, b[i]))
        dst.append(np.tile(c, a[i]))
    src, dst = np.concatenate(src), np.concatenate(dst)
    perm = rng.permutation(len(src))
    sig = np.sort(np.sqrt(a.astype(np.float64) * b))[::-1]
    return src[perm], dst[perm], np.concatenate(rows), np.concatenate(cols), sig


def _csr_expected(src, dst):
    key = np.unique(src.astype(np.int64) * N + dst.astype(np.int64))
    ip = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(key // N, minlength=N), out=ip[1:])
    return ip, (key % N).astype(np.int32)


@pytest.mark.parametrize("precision", [0, 1])
def test_large_n_bicliques(damf, precision):
    _say(f"case large_n_bicliques precision={precision} (n={N}, d={D}, {BLOCKS} bicliques)")
    src, dst, rnodes, cnodes, sig = _bicliques(11)
    eps = 1e-4
    cfg = damf.default_config(N, D, directed=True, alpha=0.15, eps=eps, oversample=10,
                              power_iters=2, seed=3, max_core_rank=64, max_side=64,
                              precision=precision)
    ctx = damf.Context.init(cfg, src, dst)
    _say(f"  init {ctx.init_info()}")
    ip, ix = ctx.export_csr()
    eip, eix = _csr_expected(src, dst)
    assert np.array_equal(ip, eip) and np.array_equal(ix, eix)
    sg = ctx.singular_values()
    err_s = np.abs(sg[:BLOCKS] - sig).max() / sig[0]
    tail = np.abs(sg[BLOCKS:]).max() / sig[0]
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([rnodes, rng.choice(N, 1000, replace=False),
                                     np.arange(N - 500, N)])).astype(np.int32)
    cols = np.unique(np.concatenate([cnodes, rng.choice(N, 1000, replace=False),
                                     np.arange(N - 500, N)])).astype(np.int32)
    X = ctx.query("X", rows).astype(np.float64)
    Y = ctx.query("Y", cols).astype(np.float64)
    # A restricted to rows x cols, from the edge list
    ri = {int(u): i for i, u in enumerate(rows)}
    ci = {int(v): j for j, v in enumerate(cols)}
    Asub = np.zeros((len(rows), len(cols)))
    for u, v in zip(src, dst):
        Asub[ri[int(u)], ci[int(v)]] = 1.0
    E = X @ Y.T - Asub
    err_p = np.linalg.norm(E) / np.linalg.norm(Asub)
    err_max = np.abs(E).max()
    rmax = ctx.residual_max()
    _say(f"  sigma err {err_s:.2e} tail {tail:.2e} product err {err_p:.2e} max {err_max:.2e} "
         f"max|R| {rmax:.2e}")
    tol = 1e-5 if precision == 0 else 1e-4
    assert np.all(np.isfinite(sg))
    assert err_s <= 1e-5 and tail <= 1e-4
    assert err_p <= tol and err_max <= 10 * tol
    assert rmax <= eps
    # one batch of inserts between biclique nodes (the first blocks hold the
    # highest ids), with the PPR push.  The inserts overlap the basis
    # (W = U^T B != 0): an edge between two isolated nodes would bring in a
    # direction orthogonal to U, which the lazy form cannot take while a
    # zero singular value is kept (F singular)
    s1 = rng.choice(rnodes, 100).astype(np.int32)
    t1 = rng.choice(cnodes, 100).astype(np.int32)
    info = ctx.update(s1, t1, np.ones(100, dtype=np.int8))
    rmax = ctx.residual_max()
    _say(f"  update: chunks {info['chunks']} push rounds {info['push_rounds']} max|R| {rmax:.2e}")
    assert rmax <= eps and np.all(np.isfinite(ctx.singular_values()))
    ip, ix = ctx.export_csr()
    eip, eix = _csr_expected(np.concatenate([src, s1]), np.concatenate([dst, t1]))
    assert np.array_equal(ip, eip) and np.array_equal(ix, eix)
    ctx.close()
