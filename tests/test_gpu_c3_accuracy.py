"""Accuracy of the precision form at its own size against the FP64 oracle.

The precision form's configuration (directed Chung-Lu 2.1, n = 4e6, m = 6e7,
d = 128) drawn on the GPU; its first update batch (2,000 edits: 95% sampler
inserts, 5% deletes of initial edges; a bounded sample of the 5,000-edit
batches the configuration streams) applied from the same initial
factorisation by the FP64 oracle, by the FP32 form and by the precision form
(bases as BF16 pairs).  Both forms are compared with the oracle by the same
checks: singular values, the product X Y^T, the leading subspaces (gap-scaled
sines), and the rows of X Y^T on a 1% row sample.

Bars: the FP32 form holds the 1e-5 bars; the precision form stores about 16
significant bits per basis element (relative 2^-17 against FP32's 2^-24), so
its bars are 1e-4, and its product error may exceed the FP32 form's (floored
at 1e-7) by at most that storage ratio, 2^7 = 128.
"""
import sys

import numpy as np
import pytest

from oracle.model import DAMFOracle
from tests._checks import (gap_scaled_ratio, product_rel_err, relative_gaps, row_product_errs,
                           subspace_sines, unit_factor)

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_precision_form_vs_oracle_at_c3_size():
    import torch
    assert torch.cuda.is_available()
    import paper_2306_08967_amd as P
    from bench import chung_lu_edges_gpu
    n, m, d, k = 4_000_000, 60_000_000, 128, 2000
    _say(f"case C3 accuracy n={n} m={m} d={d} batch={k}")
    src, dst, draw = chung_lu_edges_gpu(n, m, 2.1, 3)
    g = torch.Generator(device="cuda")
    g.manual_seed(4)
    n_del = k // 20
    s, t = draw(k - n_del)
    j = torch.randint(0, m, (n_del,), generator=g, device="cuda")
    bs = torch.cat([s.to(torch.int32), src[j]])
    bt = torch.cat([t.to(torch.int32), dst[j]])
    bo = torch.cat([torch.ones(k - n_del, dtype=torch.int8, device="cuda"),
                    torch.full((n_del,), -1, dtype=torch.int8, device="cuda")])
    perm = torch.randperm(k, generator=g, device="cuda")
    bs, bt, bo = bs[perm].contiguous(), bt[perm].contiguous(), bo[perm].contiguous()
    # which of the batch's pairs are edges of the initial graph (input
    # preparation for the oracle's small edge set: its net change only looks
    # these up)
    keys = src.to(torch.int64) * n + dst.to(torch.int64)
    bk = bs.to(torch.int64) * n + bt.to(torch.int64)
    present = torch.isin(bk, keys)
    rel_s = bs[present].cpu().numpy()
    rel_t = bt[present].cpu().numpy()
    del keys, bk
    base = dict(directed=True, alpha=1.0, oversample=10, power_iters=2, seed=3,
                max_core_rank=64, max_side=64, tau=1e-6)
    c32 = P.Context.init(P.default_config(n, d, **base), src, dst)
    st = c32.export_state()
    U0, V0, s0 = st["Ub"], st["Vb"], c32.singular_values()
    del st
    _say("  initial factors exported")
    cpr = P.Context.init_factors(P.default_config(n, d, precision=1, **base), src, dst, U0, s0, V0)
    del src, dst
    torch.cuda.empty_cache()
    orc = DAMFOracle(n, d, True, alpha=1.0, r=64, r_max=64, tau=1e-6)
    orc.init_factors(rel_s, rel_t, U0, s0, V0)
    del U0, V0
    hs, ht, ho = bs.cpu().numpy(), bt.cpu().numpy(), bo.cpu().numpy()
    io = orc.update(hs, ht, ho)
    _say(f"  oracle: {len(io['chunks'])} chunks")
    i32 = c32.update(bs, bt, bo)
    ipr = cpr.update(bs, bt, bo)
    assert i32["chunks"] == ipr["chunks"] == len(io["chunks"])
    Xo, Yo = orc.X(), orc.Y()
    gaps = relative_gaps(orc.s, d)  # the d-th gap needs s_{d+1}: not kept, so j < d only
    rows = np.random.default_rng(5).choice(n, n // 100, replace=False)
    out = {}
    for name, ctx in (("fp32", c32), ("bf16 pairs", cpr)):
        sg = ctx.singular_values()
        X, Y = ctx.query("X"), ctx.query("Y")
        err_s = float(np.abs(sg - orc.s).max() / orc.s[0])
        err_p = product_rel_err(X, Y, Xo, Yo)
        su = subspace_sines(unit_factor(X, sg), orc.U)
        sv = subspace_sines(unit_factor(Y, sg), orc.V)
        ratio = max(gap_scaled_ratio(su[:-1], gaps[:-1]), gap_scaled_ratio(sv[:-1], gaps[:-1]))
        rowe = row_product_errs(X, Y, Xo, Yo, rows)
        out[name] = (err_s, err_p, ratio, float(rowe.max()), float(np.median(rowe)))
        _say(f"  {name}: sigma {err_s:.2e} product {err_p:.2e} gap-scaled sines {ratio:.2e} "
             f"(x 1e-5/g_j) rows max {rowe.max():.2e} median {np.median(rowe):.2e}")
        del X, Y
    f32, pr = out["fp32"], out["bf16 pairs"]
    assert f32[0] <= 1e-5 and f32[1] <= 1e-5 and f32[2] <= 1.0
    assert pr[0] <= 1e-4 and pr[1] <= 1e-4 and pr[2] <= 10.0
    assert pr[1] <= 128 * max(f32[1], 1e-7)
    c32.close()
    cpr.close()
