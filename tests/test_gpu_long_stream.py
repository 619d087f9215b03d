"""Long-stream accuracy of the FP32 form (Sec. 4.1: U and V are the orthonormal
factors of the t-SVD; the lazy update keeps U = U_b P).

The benchmark's configuration scaled to n = 50,000: directed Chung-Lu (2.1),
m = 500,000, d = 128, randomized init on 90%, then 1,000 batches of 500
edits (95% preferential-attachment inserts, 5% deletes), alpha = 0.15,
eps = 1e-5, no periodic re-orthogonalisation (the library default), the
default condition limit of P (flush above 1e3).  Every 100 batches the full
U = X Sigma^(-1/2) and V are read back and ||U^T U - I||_max must stay below
1e-5 (the FP32 bar); the largest condition estimate of P and the number of
flushes are reported.  Step 4 must end every batch with max |R| <= eps.
"""
import sys

import numpy as np
import pytest

from tests._checks import orth_err, unit_factor
from workloads import chung_lu_workload

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_orthogonality_over_1000_batches():
    import torch
    assert torch.cuda.is_available()
    import paper_2306_08967_amd as P
    n, m, d, batches, k = 50_000, 500_000, 128, 1000, 500
    _say(f"case long stream n={n} m={m} d={d} batches={batches}x{k}")
    w = chung_lu_workload(n, m, 2.1, 7, batches, k, 0.95, d=d)
    cfg = P.default_config(n, d, directed=True, alpha=0.15, eps=1e-5, oversample=10,
                           power_iters=2, seed=7)
    ctx = P.Context.init(cfg, *w["init"])
    dev = [tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in b) for b in w["stream"]]
    cond_max, flushes, worst = 0.0, 0, 0.0
    for b, batch in enumerate(dev):
        info = ctx.update(*batch)
        cond_max = max(cond_max, info["p_cond"])
        flushes += info["flushed"]
        if b % 100 == 99:
            sg = ctx.singular_values()
            X, Y = ctx.query("X"), ctx.query("Y")
            eo = max(orth_err(unit_factor(X, sg)), orth_err(unit_factor(Y, sg)))
            worst = max(worst, eo)
            _say(f"  batch {b + 1}: orth {eo:.2e} cond(P) max {cond_max:.3e} flushes {flushes} "
                 f"max|R| {ctx.residual_max():.2e} sigma_1 {sg[0]:.3f} sigma_d {sg[-1]:.3f}")
            assert eo <= 1e-5
            assert ctx.residual_max() <= 1e-5
    _say(f"  worst orth {worst:.2e}, largest cond(P) {cond_max:.3e}, flushes {flushes}")
    ctx.close()
