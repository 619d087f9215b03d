"""damf_load rejects corrupt checkpoint files before it allocates or writes
anything from them (CPU only: the file checks run before any device call).

The header layout is the library's checkpoint header: 8-byte magic, five
int64 (version, n, m, batches since re-orthogonalisation, push rounds), six
int32 (d, directed, precision, ppr_on, enhance_pending, pad), one float64
(alpha); then indptr (n + 1 int64), indices (m int32), P (2 d^2 float64),
Sigma (192 float64), U_b and V_b (n d float32 each; Z_b and R too with PPR).
"""
import ctypes
import os
import struct

import numpy as np
import pytest

MAX_CORE = 192


@pytest.fixture(scope="module")
def lib():
    from paper_2306_08967_amd import _damf
    if not os.path.exists(_damf.LIB_PATH):
        from paper_2306_08967_amd import build_lib
        build_lib.build()
    return _damf.lib()


def _cfg(n, d):
    from paper_2306_08967_amd import default_config
    # alpha = 1: no PPR state in the file
    return default_config(n, d, directed=True, alpha=1.0, max_core_rank=8, max_side=8)


def _write(path, n, d, m, indptr, indices, body_m=None, truncate=0):
    hdr = b"DAMFCKP1" + struct.pack("<5q", 1, n, m, 0, 0) + struct.pack("<6i", d, 1, 0, 0, 0, 0) \
        + struct.pack("<d", 1.0)
    assert len(hdr) == 80
    body = np.asarray(indptr, np.int64).tobytes() + np.asarray(indices, np.int32).tobytes()
    body += np.zeros(2 * d * d + MAX_CORE, np.float64).tobytes()
    body += np.zeros(2 * n * d, np.float32).tobytes()
    data = hdr + body
    if truncate:
        data = data[:-truncate]
    with open(path, "wb") as f:
        f.write(data)


def _load(lib, path, cfg):
    h = ctypes.c_void_p()
    st = lib.damf_load(os.fsencode(str(path)), ctypes.byref(cfg), ctypes.byref(h))
    return st, h.value


def test_indptr_out_of_order_is_rejected(lib, tmp_path):
    # indptr = [0, 5, 1] with m = 1 passes the end checks but a row range
    # leaves [0, m]: must be refused before src is written
    n, d = 2, 4
    p = tmp_path / "bad_indptr.ckpt"
    _write(p, n, d, 1, [0, 5, 1], [0])
    st, h = _load(lib, p, _cfg(n, d))
    assert st == 1 and not h


def test_huge_edge_count_is_rejected_without_allocation(lib, tmp_path):
    n, d = 2, 4
    p = tmp_path / "huge_m.ckpt"
    _write(p, n, d, 1 << 40, [0, 0, 0], [])
    st, h = _load(lib, p, _cfg(n, d))
    assert st == 1 and not h


def test_truncated_file_is_rejected(lib, tmp_path):
    n, d = 3, 4
    p = tmp_path / "short.ckpt"
    _write(p, n, d, 2, [0, 1, 2, 2], [1, 2], truncate=12)
    st, h = _load(lib, p, _cfg(n, d))
    assert st == 1 and not h


def test_header_mismatch_is_rejected(lib, tmp_path):
    n, d = 3, 4
    p = tmp_path / "mismatch.ckpt"
    _write(p, n, d, 2, [0, 1, 2, 2], [1, 2])
    st, h = _load(lib, p, _cfg(n + 1, d))
    assert st == 1 and not h
