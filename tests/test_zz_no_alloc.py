"""damf_query_static: the query entry point that allocates nothing.

Compared with damf_query (the existing entry point) on the same context, to
the same bar (bit-identical rows: both run the same query kernel on the same
state), on two calls in a row with the second one smaller, for host and
device pointers and for X, Y and Z; plus its refusals (query larger than the
fixed scratch with host pointers, bad device id, pending Step 4).
"""
import sys

import numpy as np
import pytest

from paper_2306_08967_amd._damf import DAMF_E_INVALID_ARG, DAMF_E_OUT_OF_RANGE
from workloads import chung_lu_directed

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    import paper_2306_08967_amd as P
    n, d = 20_000, 64
    src, dst = chung_lu_directed(n, 120_000, beta=2.1, seed=41)
    cfg = P.default_config(n, d, directed=True, alpha=0.15, eps=1e-4, max_core_rank=16,
                           max_side=32)
    c = P.Context.init(cfg, src, dst)
    rng = np.random.default_rng(5)
    k = 200
    c.update(rng.integers(0, n, k).astype(np.int32), rng.integers(0, n, k).astype(np.int32),
             np.ones(k, np.int8))
    yield c
    c.close()


@pytest.mark.parametrize("which", ["X", "Y", "Z"])
def test_static_query_equals_query_host(ctx, which):
    _say(f"case static query host {which}")
    rng = np.random.default_rng(7)
    for q in (8000, 1500):  # second call smaller: stale rows must not leak
        nodes = rng.integers(0, ctx.n, q).astype(np.int32)
        ref = ctx.query(which, nodes)
        got = ctx.query_static(which, nodes)
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("which", ["X", "Z"])
def test_static_query_equals_query_device(ctx, which):
    import torch
    _say(f"case static query device {which}")
    rng = np.random.default_rng(8)
    for q in (ctx.n, 333):
        nodes = torch.from_numpy(rng.integers(0, ctx.n, q).astype(np.int32)).cuda()
        ref = torch.empty((q, ctx.d), dtype=torch.float32, device="cuda")
        got = torch.full((q, ctx.d), float("nan"), dtype=torch.float32, device="cuda")
        ctx.query(which, nodes, ref)
        ctx.query_static(which, nodes, got)
        assert torch.equal(got, ref)


def test_static_query_all_rows(ctx):
    _say("case static query all rows, device out")
    import torch
    ref = ctx.query("X")
    got = torch.empty((ctx.n, ctx.d), dtype=torch.float32, device="cuda")
    ctx.query_static("X", None, got)
    assert np.array_equal(got.cpu().numpy(), ref)


def test_static_query_refusals(ctx):
    import torch
    import paper_2306_08967_amd as P
    _say("case static query refusals")
    # host pointers: 256 + 4q + 4qd bytes must fit in 4 MiB (d = 64: q <= 16,131)
    nodes = np.zeros(17_000, np.int32)
    with pytest.raises(P.DamfError) as e:
        ctx.query_static("X", nodes)
    assert e.value.status == DAMF_E_INVALID_ARG
    bad = torch.tensor([1, ctx.n], dtype=torch.int32, device="cuda")
    out = torch.zeros((2, ctx.d), dtype=torch.float32, device="cuda")
    with pytest.raises(P.DamfError) as e:
        ctx.query_static("X", bad, out)
    assert e.value.status == DAMF_E_OUT_OF_RANGE
    assert bool((out == 0).all())
    # the context still answers afterwards
    small = np.arange(10, dtype=np.int32)
    assert np.array_equal(ctx.query_static("Y", small), ctx.query("Y", small))


def test_static_query_refuses_pending_enhancement():
    import paper_2306_08967_amd as P
    _say("case static query with Step 4 pending")
    n, d = 3000, 16
    src, dst = chung_lu_directed(n, 15_000, beta=2.1, seed=42)
    cfg = P.default_config(n, d, directed=True, alpha=0.15, eps=1e-4, max_core_rank=8,
                           max_side=16, auto_enhance=0)
    c = P.Context.init(cfg, src, dst)
    try:
        rng = np.random.default_rng(9)
        c.update(rng.integers(0, n, 50).astype(np.int32), rng.integers(0, n, 50).astype(np.int32),
                 np.ones(50, np.int8))
        nodes = np.arange(100, dtype=np.int32)
        with pytest.raises(P.DamfError) as e:
            c.query_static("Z", nodes)
        assert e.value.status == DAMF_E_INVALID_ARG
        c.enhance()
        assert np.array_equal(c.query_static("Z", nodes), c.query("Z", nodes))
    finally:
        c.close()
