"""The C-ABI library loads and exports every entry point the header declares (CPU only)."""
import glob
import os
import re
import ctypes

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "damf.h")
SERVE_HEADER = os.path.join(ROOT, "include", "damf_serve.h")
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def _declared():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(damf_[a-z_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def libdamf():
    from paper_2306_08967_amd import _damf
    if not os.path.exists(_damf.LIB_PATH):
        from paper_2306_08967_amd import build_lib
        build_lib.build()
    return _damf.lib()


def test_header_declares_core_calls():
    names = _declared()
    for must in ("damf_init", "damf_update", "damf_enhance", "damf_query", "damf_flush",
                 "damf_reorthogonalize", "damf_update_requests", "damf_server_create",
                 "damf_submit", "damf_wait", "damf_server_destroy"):
        assert must in names


def test_every_declared_symbol_is_exported(libdamf):
    for name in _declared():
        assert hasattr(libdamf, name), name
        assert isinstance(getattr(libdamf, name), ctypes._CFuncPtr)


def test_config_default_and_status_strings(libdamf):
    from paper_2306_08967_amd import _damf
    cfg = _damf.DamfConfig()
    libdamf.damf_config_default(ctypes.byref(cfg))
    assert cfg.d == 128 and cfg.directed == 1 and cfg.oversample == 10 and cfg.power_iters == 2
    assert abs(cfg.alpha - 0.15) < 1e-15 and abs(cfg.eps - 1e-5) < 1e-20
    assert cfg.max_core_rank == 64 and cfg.auto_enhance == 1
    assert libdamf.damf_status_string(0) == b"ok"
    assert libdamf.damf_status_string(2).startswith(b"node id")


def test_struct_layouts_match_header(tmp_path):
    """ctypes structs agree with the C compiler's layout of damf.h (every field offset)."""
    import shutil
    import subprocess
    from paper_2306_08967_amd import _damf
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"',
             f'#include "{SERVE_HEADER}"', "int main(void) {"]
    pairs = (("damf_config", _damf.DamfConfig), ("damf_batch_info", _damf.DamfBatchInfo),
             ("damf_init_info", _damf.DamfInitInfo),
             ("damf_request_stats", _damf.DamfRequestStats),
             ("damf_server_config", _damf.DamfServerConfig),
             ("damf_request_info", _damf.DamfRequestInfo),
             ("damf_server_stats", _damf.DamfServerStats))
    for cname, py in pairs:
        lines.append(f'printf("%zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("%zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = []
    for _, py in pairs:
        want.append(ctypes.sizeof(py))
        want += [getattr(py, f).offset for f, _ in py._fields_]
    assert got == want


def test_invalid_config_rejected_without_device(libdamf):
    """Argument checks run on the host before any HIP call."""
    from paper_2306_08967_amd import _damf
    cfg = _damf.default_config(10, d=4)
    cfg.d = 0
    h = ctypes.c_void_p()
    st = libdamf.damf_init(ctypes.byref(cfg), 0, None, None, 0, ctypes.byref(h))
    assert st == _damf.DAMF_E_INVALID_ARG and not h.value
    cfg.d = 4
    cfg.max_core_rank = 500
    st = libdamf.damf_init(ctypes.byref(cfg), 0, None, None, 0, ctypes.byref(h))
    assert st == _damf.DAMF_E_INVALID_ARG
