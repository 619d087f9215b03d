"""Checkpoint: damf_save writes a context's whole state, damf_load resumes it.

After a randomized init and three update batches the state is saved and
loaded into a second context.  The loaded state (U_b, V_b, P_U, P_V, Z_b, R,
Sigma, both CSRs) equals the saved one bit for bit, and one more batch applied
to both gives the same U_b, V_b, P, Sigma and graph bit for bit; Z_b and R may
differ by the order of Step 4's float atomics, so they are compared within
eps.  A configuration that disagrees with the file is refused.
"""
import sys

import numpy as np
import pytest

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


def _same(a, b, keys):
    sa, sb = a.export_state(), b.export_state()
    for k in keys:
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(a.singular_values(), b.singular_values())
    for t in (False, True):
        for x, y in zip(a.export_csr(transpose=t), b.export_csr(transpose=t)):
            assert np.array_equal(x, y)
    return sa, sb


@pytest.mark.parametrize("precision", [0, 1])
def test_save_load_resume(damf, precision, tmp_path):
    _say(f"case checkpoint precision={precision}")
    n, m, d, eps = 600, 6000, 16, 1e-5
    s0, t0 = chung_lu_directed(n, m, 2.1, 41)
    cfg = damf.default_config(n, d, directed=True, alpha=0.15, eps=eps, oversample=10,
                              power_iters=2, seed=4, max_core_rank=8, max_side=16,
                              precision=precision)
    a = damf.Context.init(cfg, s0, t0)
    rng = np.random.default_rng(17)
    batches = []
    for _ in range(4):
        k = 40
        batches.append((rng.integers(0, n, k).astype(np.int32), rng.integers(0, n, k).astype(np.int32),
                        rng.choice(np.array([-1, 1, 1], dtype=np.int8), k)))
    for s, t, o in batches[:3]:
        a.update(s, t, o)
    path = str(tmp_path / "ctx.damf")
    a.save(path)
    b = damf.Context.load(path, cfg)
    _same(a, b, ("Ub", "Vb", "PU", "PV", "Zb", "R"))
    assert a.residual_max() == b.residual_max()
    s, t, o = batches[3]
    a.update(s, t, o)
    b.update(s, t, o)
    sa, sb = _same(a, b, ("Ub", "Vb", "PU", "PV"))
    dz = np.abs(sa["Zb"] - sb["Zb"]).max()
    _say(f"  after one more batch: |Z_b diff| {dz:.2e}, max|R| {a.residual_max():.2e} {b.residual_max():.2e}")
    assert dz <= 2 * eps and a.residual_max() <= eps and b.residual_max() <= eps
    bad = damf.default_config(n, d + 1, directed=True, alpha=0.15, eps=eps, precision=precision)
    with pytest.raises(damf.DamfError):
        damf.Context.load(path, bad)
    a.close()
    b.close()
