"""GPU parity of the node-change path (Sec. 4.2, Theorem 1; Algorithm 2, node
branch) against the FP64 oracle, through damf_add_node.

The paper's streaming scenario: a graph starts with part of its nodes and the
rest join one at a time with their edges to nodes already present.  Here
nodes 0..n0-1 carry the initial graph (exact t-SVD, uploaded), and each later
node joins with in- and out-neighbours among the present nodes; some joining
nodes have more neighbours than r_max, so their steps are cut into pieces.
Bars as for the edge path: singular values within 1e-5 s_1, X Y^T within
1e-5 relative Frobenius error, orthonormality 1e-5, canonical CSR of A and
A^T bit-exact, and with PPR the GPU's Z_b within eps + 1e-6 max|Z| of the PPR
series of its own U_b.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle.model import DAMFOracle
from oracle.ppr import ppr_series
from tests._checks import orth_err, product_rel_err, unit_factor
from paper_2306_08967_amd._damf import DAMF_E_INVALID_ARG

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


def _initial_graph(n0, m0, seed):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n0, m0)
    t = rng.integers(0, n0, m0)
    keep = s != t
    return s[keep].astype(np.int32), t[keep].astype(np.int32)


def _assert_csr(ctx, orc):
    for tr in (False, True):
        ip, ix = ctx.export_csr(transpose=tr)
        rp, rx = orc.graph.csr(transpose=tr)
        assert np.array_equal(ip, rp) and np.array_equal(ix, rx)


def _check(ctx, orc, tag):
    sg = ctx.singular_values()
    X, Y = ctx.query("X"), ctx.query("Y")
    err_s = np.abs(sg - orc.s).max() / orc.s[0]
    err_p = product_rel_err(X, Y, orc.X(), orc.Y())
    eo = max(orth_err(unit_factor(X, sg)), orth_err(unit_factor(Y, sg)))
    _say(f"  {tag}: sigma {err_s:.2e} product {err_p:.2e} orth {eo:.2e}")
    assert err_s <= 1e-5 and err_p <= 1e-5 and eo <= 1e-5


@pytest.mark.parametrize("directed", [True, False])
def test_nodes_join_one_at_a_time(damf, directed):
    n, n0, d, r_max = 400, 300, 16, 16
    alpha, eps = 0.15, 1e-6
    _say(f"case node stream directed={directed}")
    s0, t0 = _initial_graph(n0, 3000, 71)
    orc = DAMFOracle(n, d, directed, alpha=alpha, eps=eps, r=8, r_max=r_max,
                     tau=1e-6).init_exact(s0, t0)
    cfg = damf.default_config(n, d, directed=directed, alpha=alpha, eps=eps, max_core_rank=8,
                              max_side=r_max, tau=1e-6)
    ctx = damf.Context.init_factors(cfg, s0, t0, orc.U, orc.s, orc.V)
    rng = np.random.default_rng(72)
    pieces = 0
    for j, new in enumerate(range(n0, n)):
        # 1..40 in-neighbours (more than r_max = 16 for some), 1..12 out; an
        # occasional self-loop; neighbours among the nodes already present
        k_in = int(rng.integers(1, 41)) if j % 7 else 1
        ins = rng.choice(new, k_in, replace=False).tolist()
        if j % 11 == 3:
            ins.append(new)
        outs = rng.choice(new, int(rng.integers(1, 13)), replace=False).tolist()
        info_o = orc.add_node(new, ins, outs if directed else ())
        info = ctx.add_node(new, ins, outs if directed else ())
        assert info["chunks"] == len(info_o["steps"])
        pieces += max(0, len(info_o["steps"]) - 2)
        if j % 20 == 19:
            _check(ctx, orc, f"after {j + 1} nodes")
    _check(ctx, orc, "end")
    _assert_csr(ctx, orc)
    st = ctx.export_state()
    ip, ix = ctx.export_csr()
    A = sp.csr_matrix((np.ones(len(ix)), ix, ip), shape=(n, n))
    Zs = ppr_series(A, st["Ub"], alpha)
    err = np.abs(st["Zb"] - Zs).max()
    _say(f"  |Z_b - PPR(U_b)| {err:.2e}; multi-piece steps {pieces}")
    assert err <= eps + 1e-6 * np.abs(Zs).max()
    assert pieces > 0
    ctx.close()


def test_node_with_edges_is_refused(damf):
    _say("case node refusal")
    n, d = 60, 4
    s0, t0 = _initial_graph(50, 300, 73)
    orc = DAMFOracle(n, d, True, alpha=1.0, r=4, r_max=8, tau=1e-6).init_exact(s0, t0)
    cfg = damf.default_config(n, d, directed=True, alpha=1.0, max_core_rank=4, max_side=8)
    ctx = damf.Context.init_factors(cfg, s0, t0, orc.U, orc.s, orc.V)
    before = ctx.export_state()
    node = int(s0[0])  # has out-edges
    with pytest.raises(damf.DamfError) as e:
        ctx.add_node(node, [1, 2], [3])
    assert e.value.status == DAMF_E_INVALID_ARG
    with pytest.raises(damf.DamfError):
        ctx.add_node(55, [1, 60], [])  # id out of range
    after = ctx.export_state()
    for key in ("Ub", "Vb", "PU", "PV"):
        assert np.array_equal(before[key], after[key])
    # a free slot joins normally afterwards
    orc.add_node(55, [1, 2], [3])
    ctx.add_node(55, [1, 2], [3])
    _check(ctx, orc, "after refusals")
    _assert_csr(ctx, orc)
    ctx.close()
