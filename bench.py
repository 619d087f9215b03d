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


def core_roofline(infos):
    """Roofline record of the Step 2 core-SVD kernel over the timed batches:
    counted FP64 flops (executed, and the 9 N^3-per-sweep textbook count) over
    the HIP-event time of its launches, against the chip's FP64 peak (and one
    CU's share, the kernel being one workgroup)."""
    ms = float(sum(i["ms_core_kernel"] for i in infos))
    fl = float(sum(i["core_flops"] for i in infos))
    fm = float(sum(i["core_flops_model"] for i in infos))
    n = int(sum(i["core_launches"] for i in infos))
    tf = fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    tm = fm / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    return {"kernel": "chain_core_kernel", "bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": tf / FP64_PEAK_TFLOPS, "frac_chip": tf / FP64_PEAK_TFLOPS,
            "frac_cu": tf / FP64_CU_PEAK_TFLOPS, "achieved_model_9N3": tm,
            "frac_chip_model_9N3": tm / FP64_PEAK_TFLOPS, "frac_cu_model_9N3": tm / FP64_CU_PEAK_TFLOPS,
            "ms_per_launch": ms / max(n, 1), "launches": n, "traffic": None,
            "flop_basis": "executed (Jacobi pairs x (2N dot + 6N f rotation) + 2N^2 d + 2N^2 k) and "
                          "the 9 N^3 per sweep textbook count"}


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
    ap.add_argument("--mode", choices=("update", "serve", "scaling"), default="update",
                    help="update: batches through damf_update (default); serve: the server; "
                         "scaling: per-batch and per-query time against n at a fixed batch size")
    ap.add_argument("--workload", choices=("c2", "c3", "billion"), default="c2",
                    help="c2 (default): Chung-Lu 2.1, n=1e6, m=1e7, batches of 1000 ops; c3: "
                         "Chung-Lu 2.1, n=4e6, m=6e7, precision form, batches of 5000 ops, "
                         "re-orthogonalisation every 64; billion: Chung-Lu 2.0, n=4e7, m=1e9, "
                         "precision form, batches of 100 inserts, eps=1e-6 (both generated on the GPU)")
    ap.add_argument("--billion-batch", type=int, default=100,
                    help="insertions per batch of the billion-edge form (1: single-edge updates)")
    ap.add_argument("--serve-n", type=int, default=10_000_000)
    ap.add_argument("--serve-m", type=int, default=200_000_000)
    ap.add_argument("--serve-requests", type=int, default=12000)
    ap.add_argument("--serve-sat", type=int, default=400)
    ap.add_argument("--serve-seconds", type=float, default=12.0)
    ap.add_argument("--graph-chunks", type=int, default=8,
                    help="serve: steps of at most this many chunks run as captured HIP graphs (0: off)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="serve: the server's chunk-rank tuner picks r during the warm-up")
    ap.add_argument("--extra-legs", type=int, default=1,
                    help="1: after the timed steps (untimed), link prediction on the held-out 10%%, "
                         "single-edge (k = 1) updates and node events on the same graph")
    ap.add_argument("--billion-leg", type=int, default=1,
                    help="1: run the billion-edge form (100 timed batches) in a child process and "
                         "embed its line as a sub-record")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (the reference kernel "
                         "that scales HBM byte counters) and print its size")
    return ap.parse_args()


def pct(x, q):
    return float(np.percentile(np.asarray(x), q))


def cpu_baseline(w, batches, d, r, start=None, gpu_after=None):
    """The FP64 oracle's Steps 1-3 on the first `batches` batches of the same stream.

    start: (X0, Y0, s0), the library's factors right after its initialisation; the
    oracle then starts from U = X0 / sqrt(s0), V = Y0 / sqrt(s0) (its cost does not
    depend on the values), and with gpu_after = (rows, X, Y, s), the library's rows
    after the same batches, the record carries their agreement."""
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
    if start is not None:
        X0, Y0, s0 = start
        isq = 1.0 / np.sqrt(np.asarray(s0, np.float64))
        orc.U = np.asarray(X0, np.float64) * isq[None, :]
        orc.V = np.asarray(Y0, np.float64) * isq[None, :]
        orc.s = np.asarray(s0, np.float64).copy()
    else:
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
    agreement = None
    if start is not None and gpu_after is not None:
        rows, Xg, Yg, sg = gpu_after
        Xo, Yo = orc.X()[rows], orc.Y()[rows]
        agreement = {"after_batches": int(batches), "row_sample": int(len(rows)),
                     "sigma_max_rel_err": float(np.max(np.abs(np.asarray(sg) - orc.s)) / orc.s[0]),
                     **sample_agreement((np.asarray(Xg, np.float64), np.asarray(Yg, np.float64)),
                                        (Xo, Yo))}
    return {
        "value": ops / dt,
        "unit": "edge-updates/s",
        "cores": int(threads),
        "kind": "oracle",
        "seconds": dt,
        "setup_seconds": setup,
        "sample": (f"FP64 oracle Steps 1-3 (explicit U, V; numpy/LAPACK) on the first {batches} "
                   f"batch(es) of {len(w['stream'][0][0])} ops of the same stream and graph, from "
                   + ("the library's own initial factors" if start is not None else
                      "seeded orthonormal factors of the same shape") +
                   " (its cost does not depend on their values); the oracle's Step 4 is a full PPR "
                   "series recomputation and is not timed"),
        "agreement_with_library": agreement,
    }


def fp32_accuracy(ctx, n, d):
    """State quality after the timed region, from the library's own rows: the
    orthonormality of U = X Sigma^-1/2 and V (max |U^T U - I| from d x d FP64 Grams) and
    the relative reconstruction error ||A - X Y^T||_F^2 / ||A||_F^2 (traces of the Grams
    and of X^T (A Y), A from the library's CSR)."""
    import torch
    s = torch.from_numpy(ctx.singular_values()).cuda()
    isq = 1.0 / torch.sqrt(s)
    X = torch.from_numpy(ctx.query("X")).cuda().double()
    Y = torch.from_numpy(ctx.query("Y")).cuda().double()
    GX, GY = X.T @ X, Y.T @ Y
    eye = torch.eye(d, dtype=torch.float64, device="cuda")
    orth_u = float((isq[:, None] * GX * isq[None, :] - eye).abs().max())
    orth_v = float((isq[:, None] * GY * isq[None, :] - eye).abs().max())
    ip, ix = ctx.export_csr()
    m = len(ix)
    try:
        A = torch.sparse_csr_tensor(torch.from_numpy(ip.astype(np.int64)),
                                    torch.from_numpy(ix.astype(np.int64)),
                                    torch.ones(m, dtype=torch.float64), size=(n, n)).cuda()
        cross = float((X * (A @ Y)).sum())
        del A
    except (RuntimeError, NotImplementedError):  # no sparse CSR product on this build: host
        import scipy.sparse as sp
        A = sp.csr_matrix((np.ones(m), ix, ip), shape=(n, n))
        cross = float((X.cpu().numpy() * (A @ Y.cpu().numpy())).sum())
    recon = (m - 2.0 * cross + float((GX * GY).sum())) / m
    del X, Y
    torch.cuda.empty_cache()
    return {"orth_U_max": orth_u, "orth_V_max": orth_v, "recon_rel_fro2": recon,
            "basis": "the library's X, Y, Sigma after the timed batches; A its own CSR"}


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


def rmat_requests(n, count, seed, src_dev, dst_dev, median=100.0, sigma=1.0, max_k=10000,
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
        "admitted_device_bytes_peak": st["admitted_device_bytes_peak"],
        "device_cap_bytes": st["device_cap_bytes"],
        "tuned_chunk_rank": st["tuned_chunk_rank"], "tuner_steps": st["tuner_steps"],
        "max_request_ops": int(max(len(r[0]) for r in reqs)),
        "parts_max": int(max(x["parts"] for x in infos)),
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
                         precision=args.precision, kernel_timing=0, graph_chunks=args.graph_chunks)
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

    # warm-up (with the chunk-rank tuner when asked), then saturation:
    # everything submitted at once (closed loop)
    tune = {}
    if args.autotune:
        import tempfile
        path = os.path.join(tempfile.gettempdir(), f"damf_tune_{os.getpid()}.txt")
        w0 = serve_phase(P, ctx, take(40), 0.0, 1, autotune=1, tune_cache=path,
                         max_step_requests=1)
        tune = {"tuned_chunk_rank": w0["tuned_chunk_rank"], "tuner_steps": w0["tuner_steps"]}
        log(f"tuner: chunk rank {tune['tuned_chunk_rank']} after {tune['tuner_steps']} steps")
    else:
        serve_phase(P, ctx, take(40), 0.0, 1)
    sat = serve_phase(P, ctx, take(args.serve_sat), 0.0, 2)
    log(f"saturation: {sat['ops_per_s']:.0f} ops/s, {sat['mean_requests_per_step']:.1f} req/step")
    phases = []
    # each phase offers its rate for serve_seconds; should the request pool not
    # hold that many, every phase is shortened by the same factor (the offered
    # rates are unchanged)
    fracs = (0.5, 0.8, 0.95, 0.5)
    need = sum(int(f * sat["ops_per_s"] / mean_k * args.serve_seconds) for f in fracs)
    shrink = min(1.0, (len(reqs) - at) / max(need, 1))
    if shrink < 1.0:
        log(f"request pool: phases shortened to {shrink * args.serve_seconds:.1f} s each")
    for i, frac in enumerate(fracs[:3]):
        rate = frac * sat["ops_per_s"] / mean_k
        cnt = int(rate * args.serve_seconds * shrink)
        r = serve_phase(P, ctx, take(cnt), rate, 10 + i)
        r.update(load=frac, offered_req_s=rate, offered_ops_s=rate * mean_k, coalescing=True)
        phases.append(r)
        log(f"load {frac}: p50 {r['latency_ms']['p50']:.1f} ms p99 {r['latency_ms']['p99']:.1f} ms "
            f"{r['ops_per_s']:.0f} ops/s, {r['mean_requests_per_step']:.2f} req/step")
    # the same offered load without coalescing: one request per step (a queue alone)
    rate = 0.5 * sat["ops_per_s"] / mean_k
    cnt = int(rate * args.serve_seconds * shrink)
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
                               "requests round(LogNormal(ln 100, 1)) clipped 1..10000 ops, "
                               "90% R-MAT inserts / 10% deletes of initial edges; "
                               "alpha=0.15 eps=1e-5",
                   "n": n, "m": m, "d": d, "chunk_rank": args.r,
                   "graph_chunks": args.graph_chunks, "autotune": args.autotune},
        "tuner": tune,
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
                                                "push_edges", "small_sv_columns")},
        "residual_max": ctx.residual_max(),
        "roofline": core_roofline(infos),
        "cpu_baseline": None,
        "cpu_baseline_note": "not run: the oracle keeps U and V explicitly (n x d float64, 41 GB "
                             "each at n = 4e7) and rotates all rows per chunk",
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
                                                "pushes", "small_sv_columns")},
        "accuracy": accuracy,
        "residual_max": ctx.residual_max(),
        "roofline": core_roofline(infos),
        "cpu_baseline": None,
    }
    ref.close()
    ctx.close()
    print(json.dumps(out))


def linkpred_leg(ctx, w, n, seed):
    """Link prediction (Sec. 5.2) on the benchmark graph: the 10% of its edges
    never given to the library are the positives, as many uniform non-edges
    the negatives; scores <Z[u], Y[v]> from damf_score_pairs; AUC and AP on
    up to 200,000 of each."""
    import torch
    from workloads import linkpred as lp
    rs, rt = w["heldout"]
    rng = np.random.default_rng(seed + 5)
    k = min(len(rs), 200_000)
    pick = rng.choice(len(rs), k, replace=False)
    pu, pv = rs[pick].astype(np.int32), rt[pick].astype(np.int32)
    keys = np.unique(np.concatenate([w["init"][0].astype(np.int64) * n + w["init"][1], rs.astype(np.int64) * n + rt]))
    nu, nv = lp.negative_pairs(n, k, keys, seed + 6)
    u = torch.from_numpy(np.concatenate([pu, nu])).cuda()
    v = torch.from_numpy(np.concatenate([pv, nv])).cuda()
    ctx.score_pairs(u[:1024], v[:1024])  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sc = ctx.score_pairs(u, v, "Z", "Y")
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    sc = sc.cpu().numpy()
    return {"positives": int(k), "negatives": int(k), "auc": lp.auc(sc[:k], sc[k:]),
            "ap": lp.average_precision(sc[:k], sc[k:]), "score_ms": ms,
            "pairs_per_s": 2 * k / (ms * 1e-3),
            "protocol": "positives: the benchmark graph's 10% never given to the library; "
                        "negatives: uniform non-edges; score <Z[u], Y[v]> after the timed stream"}


def k1_leg(w, src, dst, n, d, args, batches, count=300, warm=20):
    """Single-edge updates (k = 1, the paper's per-edge Theorem 2 step): the
    same graph, chunk rank 1, one edit per damf_update call taken from the
    benchmark stream; p50/p99 per update."""
    import torch
    from paper_2306_08967_amd import Context, default_config
    cfg = default_config(n, d, directed=True, alpha=0.15, eps=1e-5, oversample=10, power_iters=2,
                         seed=args.seed, max_core_rank=1, max_side=1, precision=args.precision,
                         jacobi_tol=args.jacobi_tol)
    ctx = Context.init(cfg, src, dst)
    ops = [(b[0][i:i + 1], b[1][i:i + 1], b[2][i:i + 1]) for b in batches for i in range(len(b[0]))]
    ops = ops[:warm + count]
    for o in ops[:warm]:
        ctx.update(*o)
    torch.cuda.synchronize()
    lat, cores = [], []
    t0 = time.perf_counter()
    for o in ops[warm:]:
        t = time.perf_counter()
        info = ctx.update(*o)
        lat.append(time.perf_counter() - t)
        cores.append(info["max_core"])
    T = time.perf_counter() - t0
    ctx.close()
    return {"updates": len(lat), "updates_per_s": len(lat) / T,
            "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3},
            "max_core": int(max(cores)), "chunk_rank": 1}


def node_leg(w, src, dst, n, d, args, count=300, warm=20, extra=2000):
    """Node events (Sec. 4.2, Theorem 1; the paper's streaming unit): the same
    graph in a context with `extra` free node slots; each event adds a node
    with in- and out-neighbours drawn from the stream's sampler (10 each, the
    graph's mean degree); p50/p99 per event."""
    import torch
    from paper_2306_08967_amd import Context, default_config
    n2 = n + extra
    cfg = default_config(n2, d, directed=True, alpha=0.15, eps=1e-5, oversample=10, power_iters=2,
                         seed=args.seed, max_core_rank=args.r, max_side=64, precision=args.precision,
                         jacobi_tol=args.jacobi_tol)
    ctx = Context.init(cfg, src, dst)
    rng = np.random.default_rng(args.seed + 9)
    lat, chunks = [], []
    t0 = None
    for j in range(warm + count):
        ins = rng.integers(0, n, 10).astype(np.int32)
        outs = w["init"][1][rng.integers(0, len(w["init"][1]), 10)].astype(np.int32)
        if j == warm:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        t = time.perf_counter()
        info = ctx.add_node(n + j, ins, outs)
        if j >= warm:
            lat.append(time.perf_counter() - t)
            chunks.append(info["chunks"])
    T = time.perf_counter() - t0
    ctx.close()
    return {"events": len(lat), "events_per_s": len(lat) / T,
            "latency_ms": {"p50": pct(lat, 50) * 1e3, "p99": pct(lat, 99) * 1e3},
            "edges_per_event": 20, "chunks_per_event": float(np.mean(chunks)),
            "note": "the paper reports under 10 ms per node event on 8 CPU threads (Twitter); "
                    "context, not the same graph or hardware"}


def billion_leg(args):
    """The billion-edge form in a child process (its own GPU memory), its JSON
    line embedded as a sub-record; on failure the error is recorded instead."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", "billion", "--steps", "100",
           "--warmup", "10", "--cpu-baseline", "0", "--seed", str(args.seed)]
    log("billion-edge leg (child process) ...")
    try:
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=420)
    except subprocess.TimeoutExpired:
        return {"error": "timed out after 420 s"}
    for ln in r.stderr.splitlines()[-3:]:
        log("  billion: " + ln)
    if r.returncode != 0:
        return {"error": f"exit {r.returncode}", "stderr_tail": r.stderr[-800:]}
    try:
        return json.loads(r.stdout.strip().splitlines()[-1])
    except Exception as e:  # noqa: BLE001
        return {"error": f"unparsable output: {e}"}


def scaling_main(args):
    """Sec. 4.6 claims an update cost independent of n (O(dm d^2 + d^3) per
    event) and an O(d^2) query.  Directed Chung-Lu 2.1 graphs with m = 10 n
    for n = 1e5, 1e6, 1e7 (drawn on the GPU), d = 128; batches of 1,000 edits
    (95% sampler inserts, 5% deletes of initial edges); per-batch latency, its
    Steps 1-3 and Step 4 shares, and the latency of querying 1,000 random rows
    of X and of Z."""
    import torch
    from paper_2306_08967_amd import Context, default_config
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    d, bs, K, W = args.d, 1000, args.steps, args.warmup
    rows = []
    for n in (100_000, 1_000_000, 10_000_000):
        m = 10 * n
        src, dst, draw = chung_lu_edges_gpu(n, m, 2.1, args.seed)
        g = torch.Generator(device="cuda")
        g.manual_seed(args.seed + 1)
        n_del = bs // 20
        batches = []
        for _ in range(W + K):
            s, t = draw(bs - n_del)
            j = torch.randint(0, m, (n_del,), generator=g, device="cuda")
            op = torch.cat([torch.ones(bs - n_del, dtype=torch.int8, device="cuda"),
                            torch.full((n_del,), -1, dtype=torch.int8, device="cuda")])
            batches.append((torch.cat([s.to(torch.int32), src[j]]).contiguous(),
                            torch.cat([t.to(torch.int32), dst[j]]).contiguous(), op))
        cfg = default_config(n, d, directed=True, alpha=0.15, eps=1e-5, oversample=10,
                             power_iters=2, seed=args.seed, max_core_rank=args.r, max_side=64)
        ctx = Context.init(cfg, src, dst)
        del src, dst
        for b in range(W):
            ctx.update(*batches[b])
        torch.cuda.synchronize()
        lat, infos = [], []
        for b in range(W, W + K):
            t0 = time.perf_counter()
            infos.append(ctx.update(*batches[b]))
            lat.append(time.perf_counter() - t0)
        qn = torch.from_numpy(np.random.default_rng(1).integers(0, n, 1000).astype(np.int32)).cuda()
        out = torch.empty((1000, d), device="cuda")
        qlat = {}
        for which in ("X", "Z"):
            ctx.query(which, qn, out)
            ts = []
            for _ in range(20):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.query(which, qn, out)
                ts.append(time.perf_counter() - t0)
            qlat[which] = pct(ts, 50) * 1e3
        row = {"n": n, "m": m, "batch_ms_p50": pct(lat, 50) * 1e3,
               "chain_ms_mean": float(np.mean([i["ms_chain"] for i in infos])),
               "enhance_ms_mean": float(np.mean([i["ms_enhance"] for i in infos])),
               "chunks_mean": float(np.mean([i["chunks"] for i in infos])),
               "push_edges_mean": float(np.mean([i["push_edges"] for i in infos])),
               "query_1000_rows_ms_p50": qlat}
        log(f"n={n}: {row}")
        rows.append(row)
        ctx.close()
        del batches
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "per-batch latency against n (1,000 edits, d = 128)",
                      "unit": "ms", "rows": rows, "steps": K, "warmup": W}), flush=True)


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
    if args.mode == "scaling":
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        scaling_main(args)
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
    # the oracle leg starts from the library's initial factors and is compared with its
    # rows after the same warm-up batches (untimed)
    cmp_batches = args.cpu_batches if (args.cpu_baseline and args.precision == 0
                                       and 0 < args.cpu_batches <= W) else 0
    start = gpu_after = None
    if cmp_batches:
        start = (ctx.query("X"), ctx.query("Y"), ctx.singular_values())
    for b in range(W):
        ctx.update(*batches[b])
        if cmp_batches and b + 1 == cmp_batches:
            rows = np.sort(np.random.default_rng(7).choice(n, max(1, n // 100), replace=False))
            rows_d = torch.from_numpy(rows.astype(np.int32)).cuda()
            gx = ctx.query("X", rows_d, torch.empty((len(rows), d), device="cuda")).double().cpu().numpy()
            gy = ctx.query("Y", rows_d, torch.empty((len(rows), d), device="cuda")).double().cpu().numpy()
            gpu_after = (rows, gx, gy, ctx.singular_values())
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
    core_model = tot("core_flops_model")
    core_tf_model = core_model / (core_ms * 1e-3) / 1e12 if core_ms > 0 else 0.0
    push_gbs = push_bytes / (push_ms * 1e-3) / 1e9 if push_ms > 0 else 0.0
    spmm_gbs = ii["spmm_bytes"] / (ii["ms_spmm_kernel"] * 1e-3) / 1e9 if ii["ms_spmm_kernel"] else 0.0
    kernels = {
        "chain_core_kernel": {
            "bound": "alu", "unit": "TFLOP/s", "achieved": core_tf,
            "peak": FP64_PEAK_TFLOPS, "frac": core_tf / FP64_PEAK_TFLOPS,
            "frac_chip": core_tf / FP64_PEAK_TFLOPS, "frac_cu": core_tf / FP64_CU_PEAK_TFLOPS,
            "flop_basis": "executed: Jacobi sweeps x N(N-1)/2 pairs x (2N dot + 6N f rotation, f = "
                          "share of steps whose shears ran) + 2N^2 d (H) + 2N^2 k (K), N = d + rank",
            "achieved_model_9N3": core_tf_model,
            "frac_chip_model_9N3": core_tf_model / FP64_PEAK_TFLOPS,
            "frac_cu_model_9N3": core_tf_model / FP64_CU_PEAK_TFLOPS,
            "scope": "Step 2 core SVD: one workgroup on one CU of 256 (the chunks form a serial "
                     "chain through Sigma and P); HIP events around every launch",
            "ms_per_launch": core_ms / max(core_n, 1), "launches": core_n,
            "flops_per_launch": core_flops / max(core_n, 1),
            "flops_per_launch_model_9N3": core_model / max(core_n, 1),
        },
        "chain_steps_1_3": {
            "bound": "alu", "unit": "TFLOP/s", "achieved": chain_tf,
            "peak": FP64_PEAK_TFLOPS, "frac": chain_tf / FP64_PEAK_TFLOPS,
            "frac_cu": chain_tf / FP64_CU_PEAK_TFLOPS,
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
    if dom == "chain_core_kernel":
        roofline.update({k: dk[k] for k in ("frac_chip", "frac_cu", "flop_basis", "achieved_model_9N3",
                                            "frac_chip_model_9N3", "frac_cu_model_9N3")})

    accuracy = None
    if args.precision == 0:
        accuracy = fp32_accuracy(ctx, n, d)
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
        "projection": {"p_cond_max": float(max(i["p_cond"] for i in infos)),
                       "flushes": int(tot("flushed")), "explicit_chunks": int(tot("explicit_chunks")),
                       "small_sv_columns": int(tot("small_sv_columns"))},
        "init_s": init_s,
        "init_ms": ii,
        "roofline": roofline,
        "kernels": kernels,
    }
    if args.extra_legs:
        line["link_prediction"] = linkpred_leg(ctx, w, n, args.seed)
    ctx.close()
    if args.extra_legs:
        line["single_edge_k1"] = k1_leg(w, src, dst, n, d, args, batches[W:])
        line["node_events"] = node_leg(w, src, dst, n, d, args)
    del batches, src, dst
    torch.cuda.empty_cache()
    if args.billion_leg:
        line["billion_edge"] = billion_leg(args)
    if args.cpu_baseline:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_batches, d, args.r, start=start,
                                            gpu_after=gpu_after)
        if accuracy is not None:
            accuracy["vs_oracle"] = line["cpu_baseline"]["agreement_with_library"]
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
