"""Request segments and the continuous-batching server: same result alone and in the mix.

Reading (documented with the design): a step applies its requests in admission
order, each request's net change is taken against the graph the earlier ones
leave, and no chunk mixes two requests.  Then U, Sigma, V after any
coalescing equal those of the one-by-one damf_update sequence exactly (the
chunk sequence is identical and the chain kernel is deterministic); the graph
is bit-exact; Z differs only by where Step 4 stopped, so both are within eps
of PPR(U_b) and of each other by the bound of the PPR tests.
"""
import sys
import threading
import time

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


def _requests(rng, n, count, pool, median, max_k, del_frac=0.1):
    """Requests over a small edge pool (so requests collide on edges), lognormal sizes."""
    out = []
    for _ in range(count):
        k = int(np.clip(round(rng.lognormal(np.log(median), 1.0)), 1, max_k))
        e = rng.integers(0, len(pool[0]), k)
        s, t = pool[0][e].copy(), pool[1][e].copy()
        op = np.where(rng.random(k) < del_frac, -1, 1).astype(np.int8)
        out.append((s.astype(np.int32), t.astype(np.int32), op))
    return out


def _pool(rng, n, size, loops=True):
    s = rng.integers(0, n, size).astype(np.int32)
    t = rng.integers(0, n, size).astype(np.int32)
    if loops:
        t[: size // 50] = s[: size // 50]
    return s, t


def _same_factorization(ca, cb):
    a, b = ca.export_state(), cb.export_state()
    for key in ("Ub", "Vb", "PU", "PV"):
        assert np.array_equal(a[key], b[key]), key
    assert np.array_equal(ca.singular_values(), cb.singular_values())
    for t in (False, True):
        for x, y in zip(ca.export_csr(transpose=t), cb.export_csr(transpose=t)):
            assert np.array_equal(x, y)


def _z_close(ca, cb, eps):
    za, zb = ca.query("Z").astype(np.float64), cb.query("Z").astype(np.float64)
    st = ca.export_state()
    scale = (np.abs(st["PU"]).sum(axis=0) * np.sqrt(ca.singular_values())).max()
    err = np.abs(za - zb).max()
    bound = 2 * eps * scale + 1e-6 * np.abs(zb).max()
    _say(f"  |Z mix - Z alone| {err:.2e} bound {bound:.2e}")
    assert err <= bound


@pytest.mark.parametrize("directed,alpha", [(True, 1.0), (False, 1.0), (True, 0.15)])
def test_update_requests_equals_one_by_one(damf, directed, alpha):
    _say(f"case update_requests directed={directed} alpha={alpha}")
    rng = np.random.default_rng(17)
    n, d = 300, 16
    s0, t0 = chung_lu_directed(n, 2400, 2.1, 5)
    cfg = damf.default_config(n, d, directed=directed, alpha=alpha, eps=1e-6, max_core_rank=8,
                              max_side=16, tau=1e-6, oversample=6, power_iters=2, seed=3)
    ca = damf.Context.init(cfg, s0, t0)
    cb = damf.Context.init(cfg, s0, t0)
    _same_factorization(ca, cb)
    pool = _pool(rng, n, 120)
    for rnd in range(3):
        reqs = _requests(rng, n, 14, pool, 12, 60, del_frac=0.3)
        info, per = ca.update_requests(reqs)
        alone = [cb.update(*r) for r in reqs]
        for j, (p, a) in enumerate(zip(per, alone)):
            assert p["net_entries"] == a["net_entries"], (rnd, j)
            assert p["chunks"] == a["chunks"], (rnd, j)
        assert info["chunks"] == sum(a["chunks"] for a in alone)
        _say(f"  round {rnd}: {len(reqs)} requests, {info['ops']} ops, {info['chunks']} chunks, "
             f"net {info['net_entries']}")
        _same_factorization(ca, cb)
    if alpha < 1.0:
        assert ca.residual_max() <= 1e-6 and cb.residual_max() <= 1e-6
        _z_close(ca, cb, 1e-6)
    ca.close()
    cb.close()


@pytest.mark.parametrize("overlap", [1, 0])
def test_server_same_alone_and_in_the_mix(damf, overlap):
    _say(f"case server_mix overlap={overlap}")
    rng = np.random.default_rng(23 + overlap)
    n, d, eps = 2000, 32, 1e-5
    s0, t0 = chung_lu_directed(n, 20000, 2.1, 9)
    cfg = damf.default_config(n, d, directed=True, alpha=0.15, eps=eps, max_core_rank=32,
                              max_side=64, tau=1e-6, oversample=8, power_iters=2, seed=4)
    cm = damf.Context.init(cfg, s0, t0)
    ca = damf.Context.init(cfg, s0, t0)
    pool = _pool(rng, n, 3000)
    reqs = _requests(rng, n, 90, pool, 20, 400)
    infos = {}
    with damf.Server(cm, overlap_push=overlap, start_paused=1) as srv:
        tickets = [srv.submit(*r) for r in reqs[:30]]
        assert all(t is not None for t in tickets)
        srv.resume()

        def late():
            for r in reqs[30:]:
                time.sleep(float(rng.exponential(0.002)))
                t = None
                while t is None:
                    t = srv.submit(*r)
                tickets.append(t)

        th = threading.Thread(target=late)
        th.start()
        th.join(timeout=120)
        assert not th.is_alive()
        for t in tickets:
            infos[t] = srv.wait(t, timeout_us=60_000_000)
        stats = srv.stats()
    order = sorted(infos)
    assert len(order) == len(reqs)
    steps = {infos[t]["step"] for t in order}
    coalesced = max(infos[t]["step_requests"] for t in order)
    _say(f"  {len(reqs)} requests in {len(steps)} steps (max {coalesced} per step); "
         f"p50 {stats['latency_p50_ms']:.2f} ms p99 {stats['latency_p99_ms']:.2f} ms; "
         f"push beside chain {stats['push_overlapped_ms']:.1f} ms")
    assert coalesced > 1 and stats["requests_done"] == len(reqs)
    assert all(infos[t]["status"] == 0 for t in order)
    # alone: one damf_update per request, in admission (ticket) order
    for i, t in enumerate(order):
        a = ca.update(*reqs[i])
        assert infos[t]["net_entries"] == a["net_entries"], i
        assert infos[t]["chunks"] == a["chunks"], i
    _same_factorization(cm, ca)
    assert cm.residual_max() <= eps and ca.residual_max() <= eps
    _z_close(cm, ca, eps)
    cm.close()
    ca.close()


def test_server_admission_by_memory(damf):
    _say("case server_admission")
    rng = np.random.default_rng(3)
    n, d = 200, 8
    s0, t0 = chung_lu_directed(n, 1500, 2.1, 2)
    cfg = damf.default_config(n, d, directed=True, alpha=0.15, eps=1e-5, max_core_rank=8,
                              max_side=16, oversample=4)
    ctx = damf.Context.init(cfg, s0, t0)
    pool = _pool(rng, n, 100, loops=False)
    r1, r2 = _requests(rng, n, 2, pool, 30, 30)
    # room for either request alone (9 B per op + 64 per request), not for both
    cap = 9 * max(len(r1[0]), len(r2[0])) + 64 + 10
    assert 9 * (len(r1[0]) + len(r2[0])) + 128 > cap
    with damf.Server(ctx, admit_bytes=cap, start_paused=1) as srv:
        t1 = srv.submit(*r1)
        assert t1 is not None
        assert srv.submit(*r2) is None  # over the cap while r1 is admitted
        srv.resume()
        i1 = srv.wait(t1, timeout_us=30_000_000)
        t2 = srv.submit(*r2)
        assert t2 is not None
        i2 = srv.wait(t2, timeout_us=30_000_000)
        st = srv.stats()
    assert i1["status"] == 0 and i2["status"] == 0
    assert st["busy_rejects"] == 1 and st["admitted_bytes_peak"] <= cap
    with pytest.raises(damf.DamfError):
        ctx.update(np.array([n], np.int32), np.array([0], np.int32), np.array([1], np.int8))
    ctx.close()


def test_server_request_above_step_cap(damf):
    """A 10,000-op request (the serving workload's clip) runs as parts of at
    most max_step_ops ops; the result equals damf_update on the same parts."""
    _say("case server_large_request")
    rng = np.random.default_rng(31)
    n, d = 3000, 16
    s0, t0 = chung_lu_directed(n, 24000, 2.1, 12)
    cfg = damf.default_config(n, d, directed=True, alpha=0.15, eps=1e-5, max_core_rank=16,
                              max_side=32, tau=1e-6, oversample=6, seed=5)
    cm = damf.Context.init(cfg, s0, t0)
    ca = damf.Context.init(cfg, s0, t0)
    pool = _pool(rng, n, 20000, loops=False)
    e = rng.integers(0, len(pool[0]), 10000)
    big = (pool[0][e].copy(), pool[1][e].copy(),
           np.where(rng.random(10000) < 0.1, -1, 1).astype(np.int8))
    small = _requests(rng, n, 3, pool, 50, 200)
    with damf.Server(cm, start_paused=1) as srv:
        tickets = [srv.submit(*r) for r in [small[0], big, small[1], small[2]]]
        srv.resume()
        infos = [srv.wait(t, timeout_us=120_000_000) for t in tickets]
    assert [i["status"] for i in infos] == [0, 0, 0, 0]
    assert infos[1]["parts"] == 2 and infos[1]["ops"] == 10000
    # alone: the small request, the big one in parts of 8192 and 1808, the rest
    ca.update(*small[0])
    ca.update(*(a[:8192] for a in big))
    ca.update(*(a[8192:] for a in big))
    ca.update(*small[1])
    ca.update(*small[2])
    _same_factorization(cm, ca)
    cm.close()
    ca.close()


def test_server_admission_by_device_memory(damf):
    _say("case server_device_admission")
    rng = np.random.default_rng(4)
    n, d = 200, 8
    s0, t0 = chung_lu_directed(n, 1500, 2.1, 2)
    cfg = damf.default_config(n, d, directed=True, alpha=1.0, max_core_rank=8, max_side=16,
                              oversample=4)
    ctx = damf.Context.init(cfg, s0, t0)
    pool = _pool(rng, n, 100, loops=False)
    r1, r2 = _requests(rng, n, 2, pool, 30, 30)
    # room for either request alone (24 B per op), not for both
    cap = 24 * max(len(r1[0]), len(r2[0])) + 10
    assert 24 * (len(r1[0]) + len(r2[0])) > cap
    with damf.Server(ctx, admit_device_bytes=cap, start_paused=1) as srv:
        t1 = srv.submit(*r1)
        assert t1 is not None
        assert srv.submit(*r2) is None
        srv.resume()
        srv.wait(t1, timeout_us=30_000_000)
        t2 = srv.submit(*r2)
        assert t2 is not None
        srv.wait(t2, timeout_us=30_000_000)
        st = srv.stats()
    assert st["busy_rejects"] == 1 and st["admitted_device_bytes_peak"] <= cap
    assert st["device_cap_bytes"] == cap
    ctx.close()


def test_server_chunk_rank_tuner(damf, tmp_path):
    """The tuner tries the chunk ranks, keeps one, writes the cache; a second
    server reads the cache and does not tune; every request reports the rank
    it ran with, and replaying them alone with those ranks is bit-identical."""
    _say("case server_tuner")
    rng = np.random.default_rng(41)
    n, d = 2000, 32
    s0, t0 = chung_lu_directed(n, 20000, 2.1, 9)
    cfg = damf.default_config(n, d, directed=True, alpha=1.0, max_core_rank=64, max_side=64,
                              tau=1e-6, oversample=8, seed=4)
    cm = damf.Context.init(cfg, s0, t0)
    ca = damf.Context.init(cfg, s0, t0)
    pool = _pool(rng, n, 3000)
    reqs = _requests(rng, n, 24, pool, 150, 600)
    cache = str(tmp_path / "tune.txt")
    infos = []
    with damf.Server(cm, autotune=1, tune_cache=cache, max_step_requests=1) as srv:
        tickets = [srv.submit(*r) for r in reqs]
        infos = [srv.wait(t, timeout_us=120_000_000) for t in tickets]
        st = srv.stats()
    ranks = [i["chunk_rank"] for i in infos]
    _say(f"  tuned rank {st['tuned_chunk_rank']} after {st['tuner_steps']} steps; ranks {ranks}")
    assert st["tuned_chunk_rank"] in (16, 32, 48, 64) and st["tuner_steps"] >= 16
    assert set(ranks[:16]) == {16, 32, 48, 64}
    line = open(cache).read().strip().splitlines()[-1]
    assert line.endswith(f" r={st['tuned_chunk_rank']}")
    for r, info in zip(reqs, infos):
        ca.set_chunk_rank(info["chunk_rank"])
        ca.update(*r)
    _same_factorization(cm, ca)
    # a second server: the cached rank, no tuning
    with damf.Server(cm, autotune=1, tune_cache=cache) as srv:
        t = srv.submit(*reqs[0])
        i = srv.wait(t, timeout_us=60_000_000)
        st2 = srv.stats()
    assert st2["tuner_steps"] == 0 and st2["tuned_chunk_rank"] == st["tuned_chunk_rank"]
    assert i["chunk_rank"] == st["tuned_chunk_rank"]
    cm.close()
    ca.close()
