#!/usr/bin/env python3
"""Benchmark of the DAMF update path on one MI355X.

Workload (default): directed Chung-Lu power-law graph, exponent 2.1,
n = 1,000,000 nodes, m = 10,000,000 edges, d = 128.  Randomized t-SVD init on
the first 90% of edges (p = 10, q = 2) and PPR propagation (alpha = 0.15,
eps = 1e-5); then batches of 1,000 edits (95% preferential-attachment
inserts, 5% uniform deletes).  A step is one batch through the whole path:
set-semantics batch preparation, graph edits, Steps 1-3 over every chunk and
Step 4 push until max |R| <= eps.  The batches are staged in HBM before the
timed region; each step's host call ends with the batch fully applied.

Prints one JSON line (metric, value = edge-updates/s, latency percentiles,
per-kernel rooflines, and the FP64 oracle timed on the host as cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6         # MI355X FP64 vector, whole chip
N_CU = 256
FP64_CU_PEAK_TFLOPS = FP64_PEAK_TFLOPS / N_CU  # one compute unit (single-workgroup kernel)


# Sources of the core-SVD kernel: the PMC byte counts recorded in profiles/ hold
# for the kernel built from exactly these files.
CORE_SOURCES = ["paper_2306_08967_amd/csrc/chain.hip", "paper_2306_08967_amd/csrc/jacobi_wave.h", "paper_2306_08967_amd/csrc/wave_ops.h",
                "paper_2306_08967_amd/csrc/common.h",
                "paper_2306_08967_amd/csrc/damf_internal.h"]
CORE_PMC = "profiles/pmc_chain_core_kernel_c2.md"


def core_traffic():
    """HBM bytes per core-kernel launch from the committed PMC summary, or None
    when the kernel's sources have changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, CORE_PMC)).read()
        h = hashlib.sha256()
        for f in CORE_SOURCES:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
    except OSError:
        return None
    m_t = re.search(r"^traffic_bytes_per_launch: (\d+)", text, re.M)
    m_h = re.search(r"^source_sha256: ([0-9a-f]+)", text, re.M)
    if not (m_t and m_h) or m_h.group(1) != h.hexdigest():
        return None
    return float(m_t.group(1))


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--m", type=int, default=10_000_000)
    ap.add_argument("--d", type=int, default=128)
    ap.add_argument("--batch", type=int, default=1000)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--r", type=int, default=64)
    ap.add_argument("--cpu-baseline", type=int, default=1, help="0 skips the oracle leg")
    ap.add_argument("--cpu-batches", type=int, default=1)
    ap.add_argument("--precision", type=int, default=0, choices=(0, 1),
                    help="1: the precision form (bases as BF16 pairs, BF16 MFMA rotations)")
    ap.add_argument("--jacobi-tol", type=float, default=0.0,
                    help="core SVD Jacobi tolerance of the measured context (0: the library default)")
    ap.add_argument("--mode", choices=("update", "serve"), default="update",
                    help="update: batches through damf_update (default); serve: the server")
    ap.add_argument("--workload", choices=("c2", "c3", "billion"), default="c2",
                    help="c2 (default): Chung-Lu 2.1, n=1e6, m=1e7, batches of 1000 ops; c3: "
                         "Chung-Lu 2.1, n=4e6, m=6e7, precision form, batches of 5000 ops, "
                         "re-orthogonalisation every 64; billion: Chung-Lu 2.0, n=4e7, m=1e9, "
                         "precision form, batches of 100 inserts, eps=1e-6 (both generated on the GPU)")
    ap.add_argument("--billion-batch", type=int, default=100,
                    help="insertions per batch of the billion-edge form (1: single-edge updates)")
    ap.add_argument("--serve-n", type=int, default=10_000_000)
    ap.add_argument("--serve-m", type=int, default=200_000_000)
    ap.add_argument("--serve-requests", type=int, default=6000)
    ap.add_argument("--serve-sat", type=int, default=400)
    ap.add_argument("--serve-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (the reference kernel "
                         "that scales HBM byte counters) and print its size")
    return ap.parse_args()


def pct(x, q):
    return float(np.percentile(np.asarray(x), q))


def cpu_baseline(w, batches, d, r):
    """The FP64 oracle's Steps 1-3 on the first `batches` batches of the same stream."""
    from oracle.graph import EdgeSet
    from oracle.model import DAMFOracle

    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:
        threads = os.cpu_count()
    n = w["n"]
    rng = np.random.default_rng(12345)
    orc = DAMFOracle(n, d, True, alpha=1.0, r=r, r_max=64, tau=1e-6)
    t0 = time.perf_counter()
    orc.graph = EdgeSet(n, True, *w["init"])
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    V, _ = np.linalg.qr(rng.standard_normal((n, d)))
    orc.U, orc.V = U, V
    orc.s = np.sort(rng.uniform(40.0, 260.0, d))[::-1].copy()
    setup = time.perf_counter() - t0
    ops = 0
    t0 = time.perf_counter()
    for b in range(batches):
        s, t, o = w["stream"][b]
        orc.update(s, t, o)
        ops += len(s)
    dt = time.perf_counter() - t0
    return {
        "value": ops / dt,
        "unit": "edge-updates/s",
        "cores": int(threads),
        "kind": "oracle",
        "seconds": dt,
        "setup_seconds": setup,
        "sample": (f"FP64 oracle Steps 1-3 (explicit U, V; numpy/LAPACK) on the first {batches} "
                   f"batch(es) of {len(w['stream'][0][0])} ops of the same stream and graph, from "
                   "seeded orthonormal factors of the same shape (its cost does not depend on their "
                   "values); the oracle's Step 4 is a full PPR series recomputation and is not timed"),
    }


def sample_agreement(a_xyz, r_xyz):
    """Rotation-free comparison of two factorizations on the same row sample: the relative
    Frobenius error of X Y^T (through d x d Grams) and the sine of the largest principal
    angle between the column spaces of X (and of Y)."""
    Xa, Ya = a_xyz
    Xr, Yr = r_xyz
    t1 = np.trace((Xa.T @ Xa) @ (Ya.T @ Ya))
    t2 = np.trace((Xa.T @ Xr) @ (Yr.T @ Ya))
    t3 = np.trace((Xr.T @ Xr) @ (Yr.T @ Yr))
    prod = float(np.sqrt(max(t1 - 2 * t2 + t3, 0.0)) / np.sqrt(t3))

    def sin_max(A, B):
        qa, _ = np.linalg.qr(A)
        qb, _ = np.linalg.qr(B)
        return float(np.linalg.norm(qb - qa @ (qa.T @ qb), 2))  # ||(I - Qa Qa^T) Qb||_2

    return {"product_rel_fro_err": prod, "subspace_sin_max": {"X": sin_max(Xa, Xr), "Y": sin_max(Ya, Yr)}}


def hashed_subset(keys, m, seed):
    """The first m of the distinct int64 keys in the order of a seeded multiplicative hash:
    an odd multiplier is a bijection mod 2^64, so the order has no ties and is the same in
    every process (a stand-in for a random subset in random order)."""
    import torch
    h = keys * -7046029254386353131 + (seed * 6364136223846793005) % (1 << 62)
    return keys[torch.argsort(h, stable=True)[:m]]


def rmat_edges_gpu(n, m, seed, a=0.57, b=0.19, c=0.19):
    """R-MAT edge set drawn on the GPU (torch): scale ceil(log2 n), ids >= n, self-loops and
    duplicates dropped and redrawn until m distinct edges remain, then m of them kept in hashed
    order (the same edge set in every process)."""
    import math

    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    scale = max(1, math.ceil(math.log2(n)))
    keys = torch.empty(0, dtype=torch.int64, device="cuda")
    while keys.numel() < m:
        cnt = int((m - keys.numel()) * 1.8) + 4096
        s = torch.zeros(cnt, dtype=torch.int64, device="cuda")
        t = torch.zeros_like(s)
        for _ in range(scale):
            x = torch.rand(cnt, generator=g, device="cuda")
            right = ((x >= a) & (x < a + b)) | (x >= a + b + c)
            down = x >= a + b
            s = (s << 1) | down.to(torch.int64)
            t = (t << 1) | right.to(torch.int64)
            del x, right, down
        ok = (s < n) & (t < n) & (s != t)
        k = (s[ok] << 32) | t[ok]
        del s, t, ok
        keys = torch.unique(torch.cat([keys, k]))
        del k
    keys = hashed_subset(keys, m, seed)
    return (keys >> 32).to(torch.int32), (keys & 0xFFFFFFFF).to(torch.int32)


def rmat_requests(n, count, seed, src_dev, dst_dev, median=100.0, sigma=1.0, max_k=8192,
                  ins_frac=0.9, a=0.57, b=0.19, c=0.19):
    """Request stream: sizes round(LogNormal(ln median, sigma)) clipped to [1, max_k];
    inserts drawn by R-MAT, deletes of uniformly chosen initial edges."""
    import math

    import torch
    rng = np.random.default_rng(seed)
    sizes = np.clip(np.round(rng.lognormal(np.log(median), sigma, count)), 1, max_k).astype(np.int64)
    total = int(sizes.sum())
    is_ins = rng.random(total) < ins_frac
    n_ins = int(is_ins.sum())
    scale = max(1, math.ceil(math.log2(n)))
    ins_s, ins_t = np.zeros(0, np.int64), np.zeros(0, np.int64)
    while len(ins_s) < n_ins:
        cnt = 2 * (n_ins - len(ins_s)) + 1024
        s_ = np.zeros(cnt, np.int64)
        t_ = np.zeros(cnt, np.int64)
        for _ in range(scale):
            x = rng.random(cnt)
            s_ = (s_ << 1) | (x >= a + b)
            t_ = (t_ << 1) | (((x >= a) & (x < a + b)) | (x >= a + b + c))
        ok = (s_ < n) & (t_ < n) & (s_ != t_)
        ins_s = np.concatenate([ins_s, s_[ok]])
        ins_t = np.concatenate([ins_t, t_[ok]])
    idx = torch.from_numpy(rng.integers(0, src_dev.numel(), total - n_ins)).cuda()
    del_s = src_dev[idx].cpu().numpy()
    del_t = dst_dev[idx].cpu().numpy()
    src = np.zeros(total, np.int32)
    dst = np.zeros(total, np.int32)
    op = np.where(is_ins, 1, -1).astype(np.int8)
    src[is_ins], dst[is_ins] = ins_s[:n_ins], ins_t[:n_ins]
    src[~is_ins], dst[~is_ins] = del_s, del_t
    reqs, at = [], 0
    for k in sizes:
        reqs.append((src[at:at + k], dst[at:at + k], op[at:at + k]))
        at += k
    return reqs


def serve_phase(P, ctx, reqs, rate_req_s, seed, **server_kw):
    """Open loop (rate_req_s > 0: Poisson arrivals) or closed loop (all at once)."""
    import threading
    rng = np.random.default_rng(seed)
    infos, tickets = [], []
    with P.Server(ctx, **server_kw) as srv:
        def submitter():
            t_next = time.perf_counter()
            for r in reqs:
                if rate_req_s > 0:
                    t_next += rng.exponential(1.0 / rate_req_s)
                    dt = t_next - time.perf_counter()
                    if dt > 0:
                        time.sleep(dt)
                t = srv.submit(*r)
                while t is None:
                    time.sleep(1e-4)
                    t = srv.submit(*r)
                tickets.append(t)

        th = threading.Thread(target=submitter)
        th.start()
        i = 0
        while th.is_alive() or i < len(tickets):
            if i < len(tickets):
                infos.append(srv.wait(tickets[i]))
                i += 1
            else:
                time.sleep(1e-4)
        th.join()
        st = srv.stats()
    lat = np.array([x["latency_ms"] for x in infos])
    ops = sum(x["ops"] for x in infos)
    span = (max(x["done_us"] for x in infos) - min(x["submit_us"] for x in infos)) * 1e-6
    return {
        "requests": len(infos), "ops": int(ops), "seconds": span, "ops_per_s": ops / span,
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "mean": float(lat.mean()),
                       "max": float(lat.max())},
        "steps": int(st["steps"]), "mean_requests_per_step": st["mean_requests_per_step"],
        "mean_ops_per_step": st["mean_ops_per_step"],
        "push_beside_chain_ms": st["push_overlapped_ms"],
    }


def serve_main(args):
    """Serving form: continuous batching of a Poisson stream of uneven requests."""
    import torch

    from paper_2306_08967_amd import Context, default_config
    import paper_2306_08967_amd as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n, m, d = args.serve_n, args.serve_m, args.d
    t0 = time.perf_counter()
    src, dst = rmat_edges_gpu(n, m, args.seed)
    torch.cuda.synchronize()
    log(f"serve workload: R-MAT n={n} m={m} on the GPU in {time.perf_counter() - t0:.1f}s")
    cfg = default_config(n, d, directed=True, alpha=0.15, eps=1e-5, oversample=10,
                         power_iters=2, seed=args.seed, max_core_rank=args.r, max_side=64,
                         precision=args.precision, kernel_timing=1)
    t0 = time.perf_counter()
    ctx = Context.init(cfg, src, dst)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    log(f"init {init_s:.1f}s: {ctx.init_info()}")
    reqs = rmat_requests(n, args.serve_requests, args.seed + 7, src, dst)
    del src, dst
    torch.cuda.empty_cache()
    mean_k = float(np.mean([len(r[0]) for r in reqs]))
    log(f"{len(reqs)} requests, mean {mean_k:.0f} ops")
    at = 0

    def take(cnt):
        nonlocal at
        out = reqs[at:at + cnt]
        at += cnt
        assert len(out) == cnt, "request pool exhausted"
        return out

    # warm-up, then saturation: everything submitted at once (closed loop)
    serve_phase(P, ctx, take(40), 0.0, 1)
    sat = serve_phase(P, ctx, take(args.serve_sat), 0.0, 2)
    log(f"saturation: {sat['ops_per_s']:.0f} ops/s, {sat['mean_requests_per_step']:.1f} req/step")
    phases = []
    for i, frac in enumerate((0.5, 0.8, 0.95)):
        rate = frac * sat["ops_per_s"] / mean_k
        cnt = int(rate * args.serve_seconds)
        r = serve_phase(P, ctx, take(cnt), rate, 10 + i)
        r.update(load=frac, offered_req_s=rate, offered_ops_s=rate * mean_k, coalescing=True)
        phases.append(r)
        log(f"load {frac}: p50 {r['latency_ms']['p50']:.1f} ms p99 {r['latency_ms']['p99']:.1f} ms "
            f"{r['ops_per_s']:.0f} ops/s, {r['mean_requests_per_step']:.2f} req/step")
    # the same offered load without coalescing: one request per step (a queue alone)
    rate = 0.5 * sat["ops_per_s"] / mean_k
    cnt = int(rate * args.serve_seconds)
    q = serve_phase(P, ctx, take(cnt), rate, 20, max_step_requests=1)
    q.update(load=0.5, offered_req_s=rate, offered_ops_s=rate * mean_k, coalescing=False)
    phases.append(q)
    log(f"queue only at 0.5: p50 {q['latency_ms']['p50']:.1f} ms p99 {q['latency_ms']['p99']:.1f} ms")
    ctx.close()
    line = {
        "metric": "serving edge-updates/s at saturation; p50/p99 request latency under Poisson load",
        "value": sat["ops_per_s"], "unit": "edge-updates/s", "n_gpus": 1,
        "steps": sat["steps"], "warmup": 40, "ms_per_step": sat["seconds"] * 1e3 / max(sat["steps"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "R-MAT (0.57, 0.19, 0.19) directed, ids < n, no loops/duplicates; "
                               "requests round(LogNormal(ln 100, 1)) clipped 1..8192 ops, "
                               "90% R-MAT inserts / 10% deletes of initial edges; "
                               "alpha=0.15 eps=1e-5",
                   "n": n, "m": m, "d": d, "chunk_rank": args.r},
        "saturation": sat, "load_phases": phases, "init_s": init_s,
    }
    print(json.dumps(line), flush=True)


def chung_lu_edges_gpu(n, m, beta, seed):
    """Directed Chung-Lu edge set drawn on the GPU (torch): weights (i + i0)^(-1/(beta-1))
    with i0 set so the largest expected degree is sqrt(m), independently permuted out- and
    in-labels, self-loops and duplicates dropped and redrawn until m distinct edges remain,
    then m of them kept in hashed order (the same edge set in every process).  Returns (src,
    dst) int32 device tensors and the sampler's pieces."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    from scipy.special import digamma, zeta
    gamma = 1.0 / (beta - 1.0)

    def wsum(x):  # sum_{i<n} (i + x)^-gamma in closed form (Hurwitz zeta; digamma at gamma = 1)
        if gamma == 1.0:
            return float(digamma(x + n) - digamma(x))
        if gamma > 1.0:
            return float(zeta(gamma, x) - zeta(gamma, x + n))
        return float(np.sum((np.arange(n, dtype=np.float64) + x) ** (-gamma)))

    lo, hi, target = 1e-3, float(n), m ** 0.5
    for _ in range(100):
        mid = (lo * hi) ** 0.5
        if m * mid ** (-gamma) / wsum(mid) > target:
            lo = mid
        else:
            hi = mid
    # the CDF on the host in FP64 (the same bits in every process), then to the GPU
    w = (np.arange(n, dtype=np.float64) + hi) ** (-gamma)
    cdf_h = np.cumsum(w / w.sum())
    cdf_h[-1] = 1.0
    cdf = torch.from_numpy(cdf_h).cuda()
    del w, cdf_h
    perm_out = torch.randperm(n, generator=g, device="cuda")
    perm_in = torch.randperm(n, generator=g, device="cuda")

    def draw(cnt):
        a = torch.searchsorted(cdf, torch.rand(cnt, generator=g, device="cuda", dtype=torch.float64),
                               right=True).clamp_(max=n - 1)
        b = torch.searchsorted(cdf, torch.rand(cnt, generator=g, device="cuda", dtype=torch.float64),
                               right=True).clamp_(max=n - 1)
        return perm_out[a], perm_in[b]

    keys = torch.empty(0, dtype=torch.int64, device="cuda")
    while keys.numel() < m:
        need = m - keys.numel()
        parts = []
        left = int(need * 1.05) + 4096
        while left > 0:
            c = min(left, 200_000_000)
            s, t = draw(c)
            ok = s != t
            parts.append(s[ok] * n + t[ok])
            left -= c
            del s, t, ok
        keys = torch.unique(torch.cat([keys] + parts))
        del parts
    keys = hashed_subset(keys, m, seed)
    src = (keys // n).to(torch.int32)
    dst = (keys % n).to(torch.int32)
    del keys
    return src, dst, draw


def billion_main(args):
    """Billion-edge form: one GPU holds the graph, the BF16-pair bases and the PPR state."""
    import torch

    from paper_2306_08967_amd import Context, default_config
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n, m, d, K, W, bs = 40_000_000, 1_000_000_000, 128, args.steps, args.warmup, args.billion_batch
    t0 = time.perf_counter()
    src, dst, draw = chung_lu_edges_gpu(n, m, 2.0, args.seed)
    batches = []
    for _ in range(W + K):
        s, t = draw(bs)
        batches.append((s.to(torch.int32).contiguous(), t.to(torch.int32).contiguous(),
                        torch.ones(bs, dtype=torch.int8, device="cuda")))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # hand the generator's scratch back before the library allocates
    log(f"billion workload: n={n} m={m} on the GPU in {time.perf_counter() - t0:.1f}s; "
        f"{W + K} batches of {bs} inserts")
    cfg = default_config(n, d, directed=True, alpha=0.15, eps=1e-6, oversample=10,
                         power_iters=2, seed=args.seed, max_core_rank=args.r, max_side=64,
                         precision=1, kernel_timing=1, jacobi_tol=args.jacobi_tol)
    t0 = time.perf_counter()
    ctx = Context.init(cfg, src, dst)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    del src, dst
    ii = ctx.init_info()
    log(f"init {init_s:.1f}s: graph {ii['ms_graph']:.0f} ms, rsvd {ii['ms_rsvd']:.0f} ms, "
        f"ppr {ii['ms_ppr']:.0f} ms ({ii['ppr_rounds']} rounds); device memory in use "
        f"{torch.cuda.memory_allocated() / 2**30:.1f} GiB (torch) / "
        f"{(torch.cuda.mem_get_info()[1] - torch.cuda.mem_get_info()[0]) / 2**30:.1f} GiB (device)")
    for b in range(W):
        wi = ctx.update(*batches[b])
        log(f"warmup {b + 1}/{W}: chunks {wi['chunks']} push rounds {wi['push_rounds']} "
            f"pushes {wi['pushes']}")
    torch.cuda.synchronize()
    lat, infos = [], []
    t_start = time.perf_counter()
    for b in range(W, W + K):
        t = time.perf_counter()
        infos.append(ctx.update(*batches[b]))
        lat.append(time.perf_counter() - t)
        if (b - W) % 20 == 19:
            log(f"step {b - W + 1}/{K}: last {lat[-1] * 1e3:.2f} ms")
    torch.cuda.synchronize()
    T = time.perf_counter() - t_start
    value = K * bs / T

    def mean(key):
        return float(np.mean([i[key] for i in infos]))

    out = {
        "metric": "edge-updates/s", "value": value, "unit": "edge-updates/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": T / K * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16x2", "data": "synthetic",
        "config": {"workload": f"chung-lu-2.0 n=4e7 m=1e9 d=128 batch={bs} inserts, alpha=0.15 "
                               "eps=1e-6, precision form", "n": n, "m": m, "d": d, "batch": bs},
        "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3,
                       "mean": float(np.mean(lat)) * 1e3},
        "init_s": init_s, "init_ms": ii,
        "stage_ms_mean": {k: mean(k) for k in ("ms_prepare", "ms_chain", "ms_enhance",
                                               "ms_core_kernel", "ms_push_kernel")},
        "per_batch_mean": {k: mean(k) for k in ("chunks", "sweeps", "push_rounds", "pushes",
                                                "push_edges")},
        "residual_max": ctx.residual_max(),
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def c3_main(args):
    """Precision form at its own size: directed Chung-Lu 2.1, n = 4e6, m = 6e7, d = 128,
    batches of 5,000 edits (95% inserts from the same sampler, 5% deletes of initial edges),
    FP64 re-orthogonalisation every 64 batches; then the FP32 form replays the same stream
    (untimed) for the accuracy report on a 1% row sample."""
    import torch

    from paper_2306_08967_amd import Context, default_config
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n, m, d, K, W, bs = 4_000_000, 60_000_000, 128, args.steps, args.warmup, 5000
    t0 = time.perf_counter()
    src, dst, draw = chung_lu_edges_gpu(n, m, 2.1, args.seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed + 1)
    n_del = bs // 20
    batches = []
    for _ in range(W + K):
        s, t = draw(bs - n_del)
        j = torch.randint(0, m, (n_del,), generator=g, device="cuda")
        s = torch.cat([s.to(torch.int32), src[j]])
        t = torch.cat([t.to(torch.int32), dst[j]])
        op = torch.cat([torch.ones(bs - n_del, dtype=torch.int8, device="cuda"),
                        torch.full((n_del,), -1, dtype=torch.int8, device="cuda")])
        perm = torch.randperm(bs, generator=g, device="cuda")
        batches.append((s[perm].contiguous(), t[perm].contiguous(), op[perm].contiguous()))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"c3 workload: n={n} m={m} on the GPU in {time.perf_counter() - t0:.1f}s; "
        f"{W + K} batches of {bs} ops")

    def config(precision):
        return default_config(n, d, directed=True, alpha=0.15, eps=1e-5, oversample=10,
                              power_iters=2, seed=args.seed, max_core_rank=args.r, max_side=64,
                              precision=precision, reorth_every=64, kernel_timing=1,
                              jacobi_tol=args.jacobi_tol if precision == 1 else 0.0)

    t0 = time.perf_counter()
    ctx = Context.init(config(1), src, dst)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    for b in range(W):
        ctx.update(*batches[b])
    torch.cuda.synchronize()
    lat, infos = [], []
    t_start = time.perf_counter()
    for b in range(W, W + K):
        t = time.perf_counter()
        infos.append(ctx.update(*batches[b]))
        lat.append(time.perf_counter() - t)
        if (b - W) % 20 == 19:
            log(f"step {b - W + 1}/{K}: last {lat[-1] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    T = time.perf_counter() - t_start
    value = K * bs / T

    def mean(key):
        return float(np.mean([i[key] for i in infos]))

    log("fp32 reference replay for the accuracy report ...")
    ref = Context.init(config(0), src, dst)
    for b in range(W + K):
        ref.update(*batches[b])
    rng = np.random.default_rng(0)
    rows = torch.from_numpy(np.sort(rng.choice(n, n // 100, replace=False)).astype(np.int32)).cuda()
    err, got = {}, {}
    for which in ("X", "Y", "Z"):
        a = ctx.query(which, rows, torch.empty((len(rows), d), device="cuda")).double().cpu().numpy()
        r = ref.query(which, rows, torch.empty((len(rows), d), device="cuda")).double().cpu().numpy()
        got[which] = (a, r)
        sign = np.sign((a * r).sum(axis=0))
        sign[sign == 0] = 1.0
        err[which] = float(np.linalg.norm(a * sign - r) / np.linalg.norm(r))
    s_a, s_r = ctx.singular_values(), ref.singular_values()
    accuracy = {"vs": "FP32 form on the same stream", "row_sample": int(len(rows)),
                "sigma_max_rel_err": float(np.max(np.abs(s_a - s_r)) / s_r[0]),
                "rows_rel_fro_err": err,
                **sample_agreement((got["X"][0], got["Y"][0]), (got["X"][1], got["Y"][1]))}
    out = {
        "metric": "edge-updates/s", "value": value, "unit": "edge-updates/s", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": T / K * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16x2", "data": "synthetic",
        "config": {"workload": "chung-lu-2.1 n=4e6 m=6e7 d=128 batch=5000 (95% ins / 5% del), "
                               "alpha=0.15 eps=1e-5, precision form, re-orthogonalisation every 64",
                   "n": n, "m": m, "d": d, "batch": bs, "jacobi_tol": args.jacobi_tol or 1e-8},
        "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3,
                       "mean": float(np.mean(lat)) * 1e3},
        "init_s": init_s,
        "stage_ms_mean": {k: mean(k) for k in ("ms_prepare", "ms_chain", "ms_enhance", "ms_reorth",
                                               "ms_core_kernel", "ms_push_kernel")},
        "per_batch_mean": {k: mean(k) for k in ("net_entries", "chunks", "sweeps", "push_rounds",
                                                "pushes")},
        "accuracy": accuracy,
        "residual_max": ctx.residual_max(),
        "cpu_baseline": None,
    }
    ref.close()
    ctx.close()
    print(json.dumps(out))


def copy_calibration(mib):
    """A plain device-to-device copy of known size, for scaling PMC byte counters."""
    import torch
    nbytes = mib << 20
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": nbytes, "bytes_written": nbytes,
                                           "launches": 3}}))


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.workload in ("billion", "c3"):
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        (billion_main if args.workload == "billion" else c3_main)(args)
        return
    if args.mode == "serve":
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        serve_main(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU sharding "
              "of this path is a design note, not built.", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2306_08967_amd import Context, default_config
    from workloads import chung_lu_workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n, m, d, K, W = args.n, args.m, args.d, args.steps, args.warmup
    t0 = time.perf_counter()
    w = chung_lu_workload(n, m, 2.1, args.seed, W + K, args.batch, 0.95, d=d)
    log(f"workload: n={n} m={m} batches={W + K} x {args.batch} in {time.perf_counter() - t0:.1f}s")

    src = torch.from_numpy(w["init"][0]).cuda()
    dst = torch.from_numpy(w["init"][1]).cuda()
    cfg = default_config(n, d, directed=True, alpha=0.15, eps=1e-5, oversample=10,
                         power_iters=2, seed=args.seed, max_core_rank=args.r, max_side=64,
                         precision=args.precision, kernel_timing=1, jacobi_tol=args.jacobi_tol)
    t0 = time.perf_counter()
    ctx = Context.init(cfg, src, dst)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t0
    ii = ctx.init_info()
    log(f"init {init_s:.2f}s: graph {ii['ms_graph']:.0f} ms, rsvd {ii['ms_rsvd']:.0f} ms, "
        f"ppr {ii['ms_ppr']:.0f} ms ({ii['ppr_rounds']} rounds)")
    batches = [tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in b)
               for b in w["stream"]]
    torch.cuda.synchronize()
    for b in range(W):
        ctx.update(*batches[b])
    torch.cuda.synchronize()
    lat, infos = [], []
    t_start = time.perf_counter()
    for b in range(W, W + K):
        t = time.perf_counter()
        infos.append(ctx.update(*batches[b]))
        lat.append(time.perf_counter() - t)
        if (b - W) % 50 == 49:
            log(f"step {b - W + 1}/{K}: last {lat[-1] * 1e3:.2f} ms")
    torch.cuda.synchronize()
    T = time.perf_counter() - t_start
    ops = K * args.batch
    value = ops / T

    def tot(key):
        return float(sum(i[key] for i in infos))

    chain_ms, push_ms = tot("ms_chain_kernel"), tot("ms_push_kernel")
    chain_flops, push_bytes = tot("chain_flops"), tot("push_bytes")
    n_chain = sum(1 for i in infos if i["chunks"] > 0)
    chain_tf = chain_flops / (chain_ms * 1e-3) / 1e12 if chain_ms > 0 else 0.0
    core_ms, core_flops, core_n = tot("ms_core_kernel"), tot("core_flops"), int(tot("core_launches"))
    core_tf = core_flops / (core_ms * 1e-3) / 1e12 if core_ms > 0 else 0.0
    push_gbs = push_bytes / (push_ms * 1e-3) / 1e9 if push_ms > 0 else 0.0
    spmm_gbs = ii["spmm_bytes"] / (ii["ms_spmm_kernel"] * 1e-3) / 1e9 if ii["ms_spmm_kernel"] else 0.0
    kernels = {
        "chain_core_kernel": {
            "bound": "alu", "unit": "TFLOP/s", "achieved": core_tf,
            "peak": FP64_CU_PEAK_TFLOPS, "frac": core_tf / FP64_CU_PEAK_TFLOPS,
            "scope": "Step 2 core SVD, one workgroup on one CU (FP64 vector peak / 256 CUs); "
                     "HIP events around every launch",
            "ms_per_launch": core_ms / max(core_n, 1), "launches": core_n,
            "flops_per_launch": core_flops / max(core_n, 1),
        },
        "chain_steps_1_3": {
            "bound": "alu", "unit": "TFLOP/s", "achieved": chain_tf,
            "peak": FP64_CU_PEAK_TFLOPS, "frac": chain_tf / FP64_CU_PEAK_TFLOPS,
            "scope": "all Steps 1-3 launches of a batch (front, core, back, scatter per chunk) as one span",
            "ms_per_batch": chain_ms / max(n_chain, 1), "batches": n_chain,
            "flops_per_batch": chain_flops / max(n_chain, 1),
        },
        "ppr_push": {
            "bound": "hbm", "unit": "GB/s", "achieved": push_gbs, "peak": HBM_PEAK_GBS,
            "frac": push_gbs / HBM_PEAK_GBS, "ms_total": push_ms,
            "bytes_total": push_bytes, "rounds": int(tot("push_rounds")),
        },
        "ppr_init_spmm": {
            "bound": "hbm", "unit": "GB/s", "achieved": spmm_gbs, "peak": HBM_PEAK_GBS,
            "frac": spmm_gbs / HBM_PEAK_GBS, "ms_per_launch": ii["ms_spmm_kernel"] / max(ii["ppr_rounds"], 1),
            "launches": int(ii["ppr_rounds"]),
            "bytes_per_launch": ii["spmm_bytes"] / max(ii["ppr_rounds"], 1),
        },
    }
    dom = "chain_core_kernel" if core_ms >= push_ms else "ppr_push"
    dk = kernels[dom]
    roofline = {"kernel": dom, "bound": dk["bound"], "achieved": dk["achieved"], "peak": dk["peak"],
                "unit": dk["unit"], "frac": dk["frac"],
                "traffic": core_traffic() if dom == "chain_core_kernel" else None}

    accuracy = None
    if args.precision == 1:
        # the FP32 form replays the same stream (untimed); compare on a 1% row sample
        log("fp32 reference replay for the accuracy report ...")
        cfg32 = default_config(n, d, directed=True, alpha=0.15, eps=1e-5, oversample=10,
                               power_iters=2, seed=args.seed, max_core_rank=args.r, max_side=64,
                               precision=0)
        ref = Context.init(cfg32, src, dst)
        for b in range(W + K):
            ref.update(*batches[b])
        rng = np.random.default_rng(0)
        rows = torch.from_numpy(np.sort(rng.choice(n, max(1, n // 100), replace=False)).astype(np.int32)).cuda()
        out, got = {}, {}
        for which in ("X", "Y", "Z"):
            a = ctx.query(which, rows, torch.empty((len(rows), d), device="cuda")).double().cpu().numpy()
            r = ref.query(which, rows, torch.empty((len(rows), d), device="cuda")).double().cpu().numpy()
            got[which] = (a, r)
            sign = np.sign((a * r).sum(axis=0))
            sign[sign == 0] = 1.0
            out[which] = float(np.linalg.norm(a * sign - r) / np.linalg.norm(r))
        s_a, s_r = ctx.singular_values(), ref.singular_values()
        accuracy = {"vs": "FP32 form on the same stream", "row_sample": int(len(rows)),
                    "sigma_max_rel_err": float(np.max(np.abs(s_a - s_r)) / s_r[0]),
                    "rows_rel_fro_err": out,
                    **sample_agreement((got["X"][0], got["Y"][0]), (got["X"][1], got["Y"][1]))}
        ref.close()
    del src, dst
    line = {
        "metric": "edge-updates/s",
        "value": value,
        "unit": "edge-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": T / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x2" if args.precision == 1 else "f32",
        "data": "synthetic",
        "config": {"workload": "chung-lu-2.1 n=1e6 m=1e7 d=128 batch=1000 (95% ins / 5% del), "
                               "alpha=0.15 eps=1e-5",
                   "n": n, "m": m, "d": d, "batch": args.batch, "chunk_rank": args.r,
                   "precision": "bf16 pairs" if args.precision == 1 else "fp32",
                   "jacobi_tol": args.jacobi_tol or (1e-8 if args.precision == 1 else 1e-9)},
        "accuracy": accuracy,
        "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3,
                       "mean": float(np.mean(lat)) * 1e3},
        "stage_ms_mean": {k: tot(k) / K for k in ("ms_prepare", "ms_chain", "ms_enhance",
                                                   "ms_chain_kernel", "ms_push_kernel")},
        "chain_phase_ms_mean": dict(zip(
            ["gather_project", "jacobi", "core_svd_total", "completion", "rotations",
             "p_times_f", "lu_solve_scatter", "grams_cholesky"],
            [float(np.mean([i["chain_phase_ms"][j] for i in infos])) for j in range(8)])),
        "per_batch_mean": {k: tot(k) / K for k in ("net_entries", "chunks", "sweeps",
                                                    "push_rounds", "pushes", "push_edges")},
        "init_s": init_s,
        "init_ms": ii,
        "roofline": roofline,
        "kernels": kernels,
    }
    ctx.close()
    del batches
    if args.cpu_baseline:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_batches, d, args.r)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
