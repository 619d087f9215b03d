"""Queries (Sec. 4.6: a row of X, Y or Z costs O(d^2)) through the C ABI.

- Rows from host and device node lists equal the definition
  X[u] = U_b[u] P_U Sigma^(1/2) computed in FP64 from the exported state
  (within FP32 rounding of the output, 1e-6 relative to the row scale).
- A query of more rows than one launch covers (4 x 2^16 = 262,144 rows per
  pass) takes the grid-stride loop; every row is checked.
- A device node list with an id outside [0, n) returns DAMF_E_OUT_OF_RANGE
  before any row is read, and the context stays usable.
"""
import sys

import numpy as np
import pytest

from paper_2306_08967_amd._damf import DAMF_E_OUT_OF_RANGE

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


def _random_ctx(P, n, d, seed):
    rng = np.random.default_rng(seed)
    m = 4 * n
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    U = np.linalg.qr(rng.standard_normal((n, d)))[0]
    V = np.linalg.qr(rng.standard_normal((n, d)))[0]
    S = np.sort(rng.uniform(1.0, 5.0, d))[::-1].copy()
    cfg = P.default_config(n, d, directed=True, alpha=1.0, max_core_rank=8, max_side=8)
    ctx = P.Context.init_factors(cfg, src, dst, U, S, V)
    # one batch so that P_U, P_V are no longer the identity
    k = 40
    ctx.update(rng.integers(0, n, k).astype(np.int32), rng.integers(0, n, k).astype(np.int32),
               np.ones(k, np.int8))
    return ctx, rng


def _expected(ctx, which, nodes):
    st = ctx.export_state()
    s = ctx.singular_values()
    Mb, Pm = (st["Ub"], st["PU"]) if which == "X" else (st["Vb"], st["PV"])
    return (Mb[nodes] @ Pm) * np.sqrt(s)[None, :]


def test_query_host_and_device_lists(damf):
    import torch
    _say("case query host/device n=5000 d=16")
    ctx, rng = _random_ctx(damf, 5000, 16, 31)
    nodes = rng.integers(0, 5000, 777).astype(np.int32)
    for which in ("X", "Y"):
        ref = _expected(ctx, which, nodes)
        host = ctx.query(which, nodes)
        dn = torch.from_numpy(nodes).cuda()
        dout = torch.empty((len(nodes), 16), dtype=torch.float32, device="cuda")
        ctx.query(which, dn, dout)
        dev = dout.cpu().numpy()
        scale = np.abs(ref).max()
        assert np.abs(host - ref).max() <= 1e-6 * scale
        assert np.array_equal(host, dev)
    ctx.close()


def test_query_grid_stride_covers_every_row(damf):
    import torch
    n, d = 300_000, 8
    _say(f"case query grid stride n={n} d={d}")
    ctx, rng = _random_ctx(damf, n, d, 32)
    ref = _expected(ctx, "X", np.arange(n))
    full = ctx.query("X")  # nodes = NULL: q = n rows, more than one pass
    assert np.abs(full - ref).max() <= 1e-6 * np.abs(ref).max()
    # a device list longer than one pass, in a scrambled order
    perm = rng.permutation(n).astype(np.int32)
    dout = torch.empty((n, d), dtype=torch.float32, device="cuda")
    ctx.query("X", torch.from_numpy(perm).cuda(), dout)
    assert np.array_equal(dout.cpu().numpy(), full[perm])
    ctx.close()


def test_device_list_with_bad_id_is_refused(damf):
    import torch
    _say("case query bad device id")
    ctx, rng = _random_ctx(damf, 2000, 8, 33)
    before = ctx.query("X")
    for bad in (2000, -1, 2**31 - 1):
        nodes = torch.tensor([0, 5, bad, 7], dtype=torch.int32, device="cuda")
        out = torch.full((4, 8), 7.0, dtype=torch.float32, device="cuda")
        with pytest.raises(damf.DamfError) as e:
            ctx.query("X", nodes, out)
        assert e.value.status == DAMF_E_OUT_OF_RANGE
        # nothing was written and the context still answers
        assert bool((out == 7.0).all())
    assert np.array_equal(ctx.query("X"), before)
    ctx.close()
