"""ctypes binding of libdamf (include/damf.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  Arrays may be numpy arrays (host) or torch CUDA tensors (device,
passed by data_ptr with DAMF_DEVICE_PTRS).  The binding fails loudly when the
library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdamf.so")

DAMF_OK = 0
DAMF_E_INVALID_ARG = 1
DAMF_E_OUT_OF_RANGE = 2
DAMF_E_OOM = 3
DAMF_E_DEVICE = 4
DAMF_E_NUMERIC = 5
DAMF_E_STATE = 6
DAMF_E_BUSY = 7
DAMF_E_TIMEOUT = 8
DAMF_DEVICE_PTRS = 1
DAMF_SCORE_BOTH_WAYS = 2
WHICH = {"X": 0, "Y": 1, "Z": 2}


class DamfConfig(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("d", C.c_int32),
        ("directed", C.c_int32),
        ("oversample", C.c_int32),
        ("power_iters", C.c_int32),
        ("seed", C.c_uint64),
        ("alpha", C.c_double),
        ("eps", C.c_double),
        ("max_core_rank", C.c_int32),
        ("max_side", C.c_int32),
        ("tau", C.c_double),
        ("auto_enhance", C.c_int32),
        ("reorth_every", C.c_int32),
        ("graph_slack", C.c_double),
        ("hip_stream", C.c_void_p),
        ("precision", C.c_int32),
        ("kernel_timing", C.c_int32),
        ("jacobi_tol", C.c_double),
        ("flush_cond", C.c_double),
        ("graph_chunks", C.c_int32),
        ("pad0_", C.c_int32),
    ]


class DamfBatchInfo(C.Structure):
    _fields_ = [
        ("ops", C.c_int64),
        ("net_entries", C.c_int64),
        ("chunks", C.c_int64),
        ("max_core", C.c_int32),
        ("dropped", C.c_int32),
        ("push_rounds", C.c_int64),
        ("pushes", C.c_int64),
        ("push_edges", C.c_int64),
        ("ms_prepare", C.c_double),
        ("ms_chain", C.c_double),
        ("ms_enhance", C.c_double),
        ("ms_chain_kernel", C.c_double),
        ("chain_flops", C.c_double),
        ("ms_push_kernel", C.c_double),
        ("push_bytes", C.c_double),
        ("sweeps", C.c_int64),
        ("chain_phase_ms", C.c_double * 8),
        ("ms_reorth", C.c_double),
        ("ms_core_kernel", C.c_double),
        ("core_launches", C.c_int64),
        ("core_flops", C.c_double),
        ("core_flops_model", C.c_double),
        ("p_cond", C.c_double),
        ("flushed", C.c_int32),
        ("explicit_chunks", C.c_int32),
        ("graph_launches", C.c_int64),
        ("small_sv_columns", C.c_int32),
        ("pad1_", C.c_int32),
    ]

    def as_dict(self):
        out = {k: getattr(self, k) for k, _ in self._fields_}
        out["chain_phase_ms"] = list(self.chain_phase_ms)
        return out


class DamfInitInfo(C.Structure):
    _fields_ = [
        ("ms_graph", C.c_double),
        ("ms_rsvd", C.c_double),
        ("ms_ppr", C.c_double),
        ("ppr_rounds", C.c_int64),
        ("ms_spmm_kernel", C.c_double),
        ("spmm_bytes", C.c_double),
        ("nnz", C.c_int64),
        ("qr_fallbacks", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DamfRequestStats(C.Structure):
    _fields_ = [("net_entries", C.c_int64), ("chunks", C.c_int64)]


class DamfServerConfig(C.Structure):
    _fields_ = [
        ("admit_bytes", C.c_int64),
        ("max_step_ops", C.c_int32),
        ("max_step_requests", C.c_int32),
        ("overlap_push", C.c_int32),
        ("start_paused", C.c_int32),
        ("admit_device_bytes", C.c_int64),
        ("max_request_ops", C.c_int32),
        ("autotune", C.c_int32),
        ("tune_cache", C.c_char_p),
    ]


class DamfRequestInfo(C.Structure):
    _fields_ = [
        ("ticket", C.c_int64),
        ("ops", C.c_int64),
        ("step", C.c_int64),
        ("step_requests", C.c_int32),
        ("status", C.c_int32),
        ("net_entries", C.c_int64),
        ("chunks", C.c_int64),
        ("submit_us", C.c_double),
        ("start_us", C.c_double),
        ("done_us", C.c_double),
        ("latency_ms", C.c_double),
        ("parts", C.c_int32),
        ("chunk_rank", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DamfServerStats(C.Structure):
    _fields_ = [
        ("requests_done", C.c_int64),
        ("ops_done", C.c_int64),
        ("steps", C.c_int64),
        ("busy_rejects", C.c_int64),
        ("admitted_bytes_peak", C.c_int64),
        ("elapsed_s", C.c_double),
        ("ops_per_s", C.c_double),
        ("latency_p50_ms", C.c_double),
        ("latency_p99_ms", C.c_double),
        ("latency_mean_ms", C.c_double),
        ("latency_max_ms", C.c_double),
        ("mean_requests_per_step", C.c_double),
        ("mean_ops_per_step", C.c_double),
        ("push_overlapped_ms", C.c_double),
        ("admitted_device_bytes_peak", C.c_int64),
        ("device_cap_bytes", C.c_int64),
        ("tuned_chunk_rank", C.c_int32),
        ("pad_", C.c_int32),
        ("tuner_steps", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DamfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"damf status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libdamf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2306_08967_amd.build_lib`")
    L = C.CDLL(LIB_PATH)
    p = C.c_void_p
    i32p = C.POINTER(C.c_int32)
    L.damf_config_default.argtypes = [C.POINTER(DamfConfig)]
    L.damf_config_default.restype = None
    L.damf_init.argtypes = [C.POINTER(DamfConfig), C.c_int64, p, p, C.c_int32, C.POINTER(p)]
    L.damf_init_factors.argtypes = [C.POINTER(DamfConfig), C.c_int64, p, p, p, p, p, C.c_int32,
                                    C.POINTER(p)]
    L.damf_update.argtypes = [p, C.c_int64, p, p, p, C.c_int32, C.POINTER(DamfBatchInfo)]
    L.damf_update_requests.argtypes = [p, C.c_int32, C.POINTER(C.c_int64), p, p, p, C.c_int32,
                                       C.POINTER(DamfBatchInfo), C.POINTER(DamfRequestStats)]
    L.damf_enhance.argtypes = [p]
    L.damf_set_chunk_rank.argtypes = [p, C.c_int32]
    L.damf_add_node.argtypes = [p, C.c_int32, C.c_int64, p, C.c_int64, p, C.POINTER(DamfBatchInfo)]
    L.damf_server_config_default.argtypes = [C.POINTER(DamfServerConfig)]
    L.damf_server_config_default.restype = None
    L.damf_server_create.argtypes = [p, C.POINTER(DamfServerConfig), C.POINTER(p)]
    L.damf_submit.argtypes = [p, C.c_int64, p, p, p, C.POINTER(C.c_int64)]
    L.damf_wait.argtypes = [p, C.c_int64, C.c_int64, C.POINTER(DamfRequestInfo)]
    L.damf_server_resume.argtypes = [p]
    L.damf_server_get_stats.argtypes = [p, C.POINTER(DamfServerStats)]
    L.damf_server_destroy.argtypes = [p]
    L.damf_server_destroy.restype = None
    for name in ("damf_update_requests", "damf_server_create", "damf_submit", "damf_wait",
                 "damf_server_resume", "damf_server_get_stats"):
        getattr(L, name).restype = C.c_int
    L.damf_flush.argtypes = [p]
    L.damf_reorthogonalize.argtypes = [p]
    L.damf_query.argtypes = [p, C.c_int, C.c_int64, p, p, C.c_int32]
    L.damf_query_static.argtypes = [p, C.c_int, C.c_int64, p, p, C.c_int32]
    L.damf_singular_values.argtypes = [p, p]
    L.damf_score_pairs.argtypes = [p, C.c_int, C.c_int, C.c_int64, p, p, p, C.c_int32]
    L.damf_export_csr.argtypes = [p, C.c_int32, p, p, C.POINTER(C.c_int64)]
    L.damf_export_state.argtypes = [p, p, p, p, p, p, p]
    L.damf_residual_max.argtypes = [p, C.POINTER(C.c_double)]
    L.damf_get_init_info.argtypes = [p, C.POINTER(DamfInitInfo)]
    L.damf_sync.argtypes = [p]
    L.damf_save.argtypes = [p, C.c_char_p]
    L.damf_load.argtypes = [C.c_char_p, C.POINTER(DamfConfig), C.POINTER(C.c_void_p)]
    L.damf_destroy.argtypes = [p]
    L.damf_destroy.restype = None
    L.damf_last_error.argtypes = [p]
    L.damf_last_error.restype = C.c_char_p
    L.damf_status_string.argtypes = [C.c_int]
    L.damf_status_string.restype = C.c_char_p
    for name in ("damf_init", "damf_init_factors", "damf_update", "damf_add_node", "damf_enhance",
                 "damf_set_chunk_rank",
                 "damf_flush",
                 "damf_reorthogonalize", "damf_query", "damf_query_static",
                 "damf_singular_values", "damf_score_pairs", "damf_export_csr", "damf_export_state",
                 "damf_residual_max", "damf_sync", "damf_get_init_info", "damf_save", "damf_load"):
        getattr(L, name).restype = C.c_int
    del i32p
    _lib = L
    return L


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype):
    """(pointer, is_device, keepalive) for a numpy array or torch tensor."""
    if x is None:
        return None, False, None
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(x.data_ptr()), x.is_cuda, x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data_as(C.c_void_p), False, a


def default_config(n, d=128, directed=True, **kw):
    cfg = DamfConfig()
    lib().damf_config_default(C.byref(cfg))
    cfg.n = int(n)
    cfg.d = int(d)
    cfg.directed = 1 if directed else 0
    for k, v in kw.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


class Context:
    """A DAMF state on the GPU (owns a damf_ctx)."""

    def __init__(self, handle, cfg):
        self._h = handle
        self.cfg = cfg
        self.n = cfg.n
        self.d = cfg.d

    def _check(self, st):
        if st != DAMF_OK:
            msg = lib().damf_last_error(self._h).decode() if self._h else ""
            raise DamfError(st, msg or lib().damf_status_string(st).decode())

    @staticmethod
    def _create(fn, cfg, *args):
        h = C.c_void_p()
        st = fn(C.byref(cfg), *args, C.byref(h))
        if st != DAMF_OK:
            raise DamfError(st, lib().damf_status_string(st).decode())
        return Context(h, cfg)

    @classmethod
    def init(cls, cfg, src, dst):
        ps, dev, ka1 = _ptr(src, np.int32)
        pd, _, ka2 = _ptr(dst, np.int32)
        m = len(src)
        return cls._create(lib().damf_init, cfg, C.c_int64(m), ps, pd,
                           C.c_int32(DAMF_DEVICE_PTRS if dev else 0))

    @classmethod
    def init_factors(cls, cfg, src, dst, U, S, V):
        ps, dev, ka1 = _ptr(src, np.int32)
        pd, _, ka2 = _ptr(dst, np.int32)
        U = np.ascontiguousarray(U, dtype=np.float64)
        S = np.ascontiguousarray(S, dtype=np.float64)
        V = np.ascontiguousarray(V, dtype=np.float64)
        return cls._create(lib().damf_init_factors, cfg, C.c_int64(len(src)), ps, pd,
                           U.ctypes.data_as(C.c_void_p), S.ctypes.data_as(C.c_void_p),
                           V.ctypes.data_as(C.c_void_p),
                           C.c_int32(DAMF_DEVICE_PTRS if dev else 0))

    def update(self, src, dst, op):
        ps, dev, ka1 = _ptr(src, np.int32)
        pd, _, ka2 = _ptr(dst, np.int32)
        po, _, ka3 = _ptr(op, np.int8)
        info = DamfBatchInfo()
        self._check(lib().damf_update(self._h, C.c_int64(len(src)), ps, pd, po,
                                      C.c_int32(DAMF_DEVICE_PTRS if dev else 0), C.byref(info)))
        return info.as_dict()

    def update_requests(self, requests):
        """Apply [(src, dst, op), ...] as one step; returns (batch info, per-request stats)."""
        nreq = len(requests)
        sizes = (C.c_int64 * nreq)(*[len(r[0]) for r in requests])
        if requests and _is_torch(requests[0][0]):
            import torch
            src = torch.cat([r[0] for r in requests]).contiguous()
            dst = torch.cat([r[1] for r in requests]).contiguous()
            op = torch.cat([r[2] for r in requests]).contiguous()
        else:
            src = np.concatenate([np.asarray(r[0], dtype=np.int32) for r in requests])
            dst = np.concatenate([np.asarray(r[1], dtype=np.int32) for r in requests])
            op = np.concatenate([np.asarray(r[2], dtype=np.int8) for r in requests])
        ps, dev, ka1 = _ptr(src, np.int32)
        pd, _, ka2 = _ptr(dst, np.int32)
        po, _, ka3 = _ptr(op, np.int8)
        info = DamfBatchInfo()
        per = (DamfRequestStats * nreq)()
        self._check(lib().damf_update_requests(self._h, C.c_int32(nreq), sizes, ps, pd, po,
                                               C.c_int32(DAMF_DEVICE_PTRS if dev else 0),
                                               C.byref(info), per))
        return info.as_dict(), [dict(net_entries=x.net_entries, chunks=x.chunks) for x in per]

    def add_node(self, node, in_nbrs, out_nbrs=()):
        """Node change (damf_add_node): `node` joins with in-edges (v, node) and
        out-edges (node, w); undirected graphs take the neighbours in in_nbrs."""
        a = np.ascontiguousarray(np.asarray(in_nbrs, dtype=np.int32))
        b = np.ascontiguousarray(np.asarray(out_nbrs, dtype=np.int32))
        info = DamfBatchInfo()
        self._check(lib().damf_add_node(self._h, C.c_int32(int(node)), C.c_int64(len(a)),
                                        a.ctypes.data_as(C.c_void_p), C.c_int64(len(b)),
                                        b.ctypes.data_as(C.c_void_p), C.byref(info)))
        return info.as_dict()

    def set_chunk_rank(self, r):
        """damf_set_chunk_rank: chunk rank r for the batches that follow."""
        self._check(lib().damf_set_chunk_rank(self._h, C.c_int32(int(r))))

    def enhance(self):
        self._check(lib().damf_enhance(self._h))

    def flush(self):
        self._check(lib().damf_flush(self._h))

    def reorthogonalize(self):
        self._check(lib().damf_reorthogonalize(self._h))

    def query(self, which, nodes=None, out=None):
        if nodes is None:
            q = self.n
            pn = None
            dev = False
        else:
            pn, dev, ka = _ptr(nodes, np.int32)
            q = len(nodes)
        if out is None:
            out = np.empty((q, self.d), dtype=np.float32)
        po, odev, kb = _ptr(out, np.float32)
        if dev != odev and nodes is not None:
            raise ValueError("nodes and out must both be host or both be device")
        self._check(lib().damf_query(self._h, WHICH[which], C.c_int64(q), pn, po,
                                     C.c_int32(DAMF_DEVICE_PTRS if odev else 0)))
        return out

    def query_static(self, which, nodes=None, out=None):
        """damf_query_static: as query(), with no device allocation."""
        if nodes is None:
            q = self.n
            pn = None
            dev = False
        else:
            pn, dev, ka = _ptr(nodes, np.int32)
            q = len(nodes)
        if out is None:
            out = np.empty((q, self.d), dtype=np.float32)
        po, odev, kb = _ptr(out, np.float32)
        if dev != odev and nodes is not None:
            raise ValueError("nodes and out must both be host or both be device")
        self._check(lib().damf_query_static(self._h, WHICH[which], C.c_int64(q), pn, po,
                                            C.c_int32(DAMF_DEVICE_PTRS if odev else 0)))
        return out

    def score_pairs(self, u, v, which_a="Z", which_b="Y", both_ways=False, out=None):
        """damf_score_pairs: <A[u_i], B[v_i]> (max over both directions with both_ways)."""
        pu, dev, ka = _ptr(u, np.int32)
        pv, dev2, kb = _ptr(v, np.int32)
        if dev != dev2:
            raise ValueError("u and v must both be host or both be device")
        q = len(u)
        if out is None:
            if dev:
                import torch
                out = torch.empty(q, dtype=torch.float32, device=u.device)
            else:
                out = np.empty(q, dtype=np.float32)
        po, odev, kc = _ptr(out, np.float32)
        flags = (DAMF_DEVICE_PTRS if dev else 0) | (DAMF_SCORE_BOTH_WAYS if both_ways else 0)
        self._check(lib().damf_score_pairs(self._h, WHICH[which_a], WHICH[which_b], C.c_int64(q),
                                           pu, pv, po, C.c_int32(flags)))
        return out

    def singular_values(self):
        s = np.empty(self.d, dtype=np.float64)
        self._check(lib().damf_singular_values(self._h, s.ctypes.data_as(C.c_void_p)))
        return s

    def export_csr(self, transpose=False):
        m = C.c_int64()
        self._check(lib().damf_export_csr(self._h, int(transpose), None, None, C.byref(m)))
        indptr = np.empty(self.n + 1, dtype=np.int64)
        indices = np.empty(max(m.value, 1), dtype=np.int32)
        self._check(lib().damf_export_csr(self._h, int(transpose),
                                          indptr.ctypes.data_as(C.c_void_p),
                                          indices.ctypes.data_as(C.c_void_p), C.byref(m)))
        return indptr, indices[:m.value]

    def export_state(self):
        n, d = self.n, self.d
        Ub = np.empty((n, d)); Vb = np.empty((n, d)); Zb = np.empty((n, d)); R = np.empty((n, d))
        PU = np.empty((d, d)); PV = np.empty((d, d))
        args = [a.ctypes.data_as(C.c_void_p) for a in (Ub, Vb, PU, PV, Zb, R)]
        self._check(lib().damf_export_state(self._h, *args))
        return dict(Ub=Ub, Vb=Vb, PU=PU, PV=PV, Zb=Zb, R=R)

    def init_info(self):
        info = DamfInitInfo()
        self._check(lib().damf_get_init_info(self._h, C.byref(info)))
        return info.as_dict()

    def residual_max(self):
        v = C.c_double()
        self._check(lib().damf_residual_max(self._h, C.byref(v)))
        return v.value

    def sync(self):
        self._check(lib().damf_sync(self._h))

    def save(self, path):
        """Write the whole state to `path` (damf_save)."""
        self._check(lib().damf_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path, cfg):
        """A context from a damf_save file; cfg must match its n, d, directed,
        precision and alpha."""
        h = C.c_void_p()
        st = lib().damf_load(os.fsencode(path), C.byref(cfg), C.byref(h))
        if st != DAMF_OK:
            raise DamfError(st, lib().damf_status_string(st).decode())
        return Context(h, cfg)

    def close(self):
        if self._h:
            lib().damf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def server_config(**kw):
    cfg = DamfServerConfig()
    lib().damf_server_config_default(C.byref(cfg))
    for k, v in kw.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        if k == "tune_cache" and isinstance(v, str):
            v = os.fsencode(v)
        setattr(cfg, k, v)
    return cfg


class Server:
    """Continuous-batching update server on a Context (include/damf_serve.h).

    While it runs, the context belongs to the server: call no Context method
    until close().
    """

    def __init__(self, ctx, **kw):
        self.ctx = ctx
        cfg = server_config(**kw)
        h = C.c_void_p()
        st = lib().damf_server_create(ctx._h, C.byref(cfg), C.byref(h))
        if st != DAMF_OK:
            raise DamfError(st, lib().damf_status_string(st).decode())
        self._h = h

    def submit(self, src, dst, op):
        """Admit a request; returns its ticket, or None when the admission cap is reached."""
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        op = np.ascontiguousarray(op, dtype=np.int8)
        t = C.c_int64()
        st = lib().damf_submit(self._h, C.c_int64(len(src)), src.ctypes.data_as(C.c_void_p),
                               dst.ctypes.data_as(C.c_void_p), op.ctypes.data_as(C.c_void_p),
                               C.byref(t))
        if st == DAMF_E_BUSY:
            return None
        if st != DAMF_OK:
            raise DamfError(st, lib().damf_status_string(st).decode())
        return t.value

    def wait(self, ticket, timeout_us=-1):
        info = DamfRequestInfo()
        st = lib().damf_wait(self._h, C.c_int64(ticket), C.c_int64(timeout_us), C.byref(info))
        if st != DAMF_OK:
            raise DamfError(st, lib().damf_status_string(st).decode())
        return info.as_dict()

    def resume(self):
        st = lib().damf_server_resume(self._h)
        if st != DAMF_OK:
            raise DamfError(st, lib().damf_status_string(st).decode())

    def stats(self):
        out = DamfServerStats()
        st = lib().damf_server_get_stats(self._h, C.byref(out))
        if st != DAMF_OK:
            raise DamfError(st, lib().damf_status_string(st).decode())
        return out.as_dict()

    def close(self):
        if self._h:
            lib().damf_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
