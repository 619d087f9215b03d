"""The precision form (bases as BF16 pairs, BF16 MFMA rotations, FP64 core) against the oracle.

Each basis element is stored as hi = bf16(x) and lo = bf16(x - hi): its
relative representation error is at most 2^-8 * 2^-8 = 2^-16 (1.5e-5), against
2^-24 for FP32.  Rounding errors of independent entries average out in the
Frobenius norm (relative ~ 2^-16 / sqrt(3), 9e-6) and a row touched t times
adds about sqrt(t) more; the singular values are FP64 state fed only through
projections of stored rows.  The bounds below (1e-4 on the embedding product
and orthogonality, 1e-5 on sigma) allow ~10x that estimate.  The FP32 form's
errors on the same stream are printed beside them.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.factor import tsvd_randomized
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


def test_precision_c1_parity(damf):
    _say("case precision_c1")
    w = c1_workload()
    orc = DAMFOracle(w["n"], w["d"], False, alpha=1.0, r=32, r_max=64, tau=1e-6).init_exact(*w["init"])
    # (precision form, core Jacobi tolerance; 0 = the default: 1e-9 for FP32
    # bases, 1e-8 for the precision form)
    forms = ((0, 0.0), (1, 1e-9), (1, 0.0), (1, 1e-7))
    ctxs = {}
    for prec, jtol in forms:
        cfg = damf.default_config(orc.n, orc.d, directed=False, alpha=1.0, max_core_rank=32,
                                  max_side=64, tau=1e-6, precision=prec, jacobi_tol=jtol)
        ctxs[(prec, jtol)] = damf.Context.init_factors(cfg, *w["init"], orc.U, orc.s, orc.V)
    errs = {}
    for b, (s, t, op) in enumerate(w["stream"]):
        orc.update(s, t, op)
        for prec, ctx in ctxs.items():
            ctx.update(s, t, op)
    for prec, ctx in ctxs.items():
        sg = ctx.singular_values()
        X, Y = ctx.query("X"), ctx.query("Y")
        errs[prec] = (np.max(np.abs(sg - orc.s)) / orc.s[0], product_rel_err(X, Y, orc.X(), orc.Y()),
                      max(orth_err(unit_factor(X, sg)), orth_err(unit_factor(Y, sg))))
        _say(f"  precision {prec[0]} jacobi_tol {prec[1]:g}: sigma err {errs[prec][0]:.2e} "
             f"product err {errs[prec][1]:.2e} orth {errs[prec][2]:.2e}")
        ctx.close()
    assert errs[(0, 0.0)][0] <= 1e-5 and errs[(0, 0.0)][1] <= 1e-5
    for form in forms[1:]:
        assert errs[form][0] <= 1e-5 and errs[form][1] <= 1e-5 and errs[form][2] <= 1e-4, form


def test_precision_rsvd_and_ppr_invariant(damf):
    """Randomized init and PPR propagation with BF16-pair bases."""
    _say("case precision_init")
    n, m, d, p, q, seed, alpha = 3000, 30000, 16, 10, 2, 5, 0.15
    s0, t0 = chung_lu_directed(n, m, 2.1, 31)
    A = sp.csr_matrix((np.ones(m), (s0, t0)), shape=(n, n))
    U, s, V = tsvd_randomized(A, d, p, q, seed)
    cfg = damf.default_config(n, d, directed=True, alpha=alpha, eps=1e-6, oversample=p,
                              power_iters=q, seed=seed, precision=1)
    ctx = damf.Context.init(cfg, s0, t0)
    sg = ctx.singular_values()
    X, Y = ctx.query("X"), ctx.query("Y")
    err_s = np.abs(sg - s).max() / s[0]
    err_p = product_rel_err(X, Y, U * np.sqrt(s), V * np.sqrt(s))
    st = ctx.export_state()
    deg = np.asarray(A.sum(axis=1)).ravel()
    Pm = sp.diags(np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0.0)) @ A
    inv = np.abs((st["Ub"] - st["R"]) - (st["Zb"] - (1 - alpha) * (Pm @ st["Zb"])) / alpha).max()
    scale = np.abs(st["Ub"]).max()
    _say(f"  sigma err {err_s:.2e} product err {err_p:.2e} invariant {inv:.2e} (|U_b| {scale:.2e})")
    assert err_s <= 1e-5  # sigma is FP64 state: the split only enters through stored U_b, V_b
    assert err_p <= 1e-4
    # Z_b and R are FP32; U_b carries <= 2^-16 relative error, amplified by 1/alpha
    assert inv <= 3e-4 * max(scale, 1e-12)
    ctx.close()


@pytest.mark.parametrize("n,d", [(2500, 64), (5001, 128), (1500, 13)])
def test_precision_reorth_bf16_mfma(damf, n, d):
    """Re-orthogonalisation rotates the BF16-pair bases with BF16 MFMA (three products).
    n = 5001 leaves a ragged last row block after several blocks per workgroup;
    d = 13 pads the 16-wide MFMA tiles and moves rows 4 bytes at a time."""
    _say(f"case precision_reorth n={n} d={d}")
    rng = np.random.default_rng(3)
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    V, _ = np.linalg.qr(rng.standard_normal((n, d)))
    U = U @ (np.eye(d) + 1e-3 * rng.standard_normal((d, d)))
    V = V @ (np.eye(d) + 1e-3 * rng.standard_normal((d, d)))
    s = np.sort(rng.uniform(2.0, 30.0, d))[::-1].copy()
    s0, t0 = chung_lu_directed(n, 8 * n, 2.1, 33)
    cfg = damf.default_config(n, d, directed=True, alpha=1.0, max_core_rank=8, max_side=16,
                              tau=1e-6, precision=1)
    ctx = damf.Context.init_factors(cfg, s0, t0, U, s, V)
    for _ in range(3):
        k = 40
        src, dst = rng.integers(0, n, k), rng.integers(0, n, k)
        ctx.update(src, dst, rng.choice(np.array([-1, 1, 1], dtype=np.int8), k))
    st = ctx.export_state()
    Ue, Ve = st["Ub"] @ st["PU"], st["Vb"] @ st["PV"]
    se = ctx.singular_values()
    Uo, so, Vo = reorthogonalize(Ue, se, Ve)
    ctx.reorthogonalize()
    st2 = ctx.export_state()
    sg = ctx.singular_values()
    err_s = np.max(np.abs(sg - so)) / so[0]
    err_p = product_rel_err(st2["Ub"] * sg, st2["Vb"], Uo * so, Vo)
    e1 = max(orth_err(st2["Ub"]), orth_err(st2["Vb"]))
    _say(f"  sigma err {err_s:.2e} product err {err_p:.2e} orth after {e1:.2e}")
    # sigma comes from FP64 Grams of the stored bases; the rotated bases carry
    # the BF16-pair representation error (2^-16) and the MFMA's FP32 sums
    assert err_s <= 1e-6 and err_p <= 1e-4 and e1 <= 2e-4
    ctx.close()
