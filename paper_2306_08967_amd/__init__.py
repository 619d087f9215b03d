"""DAMF (arXiv 2306.08967) on MI355X: dynamic adjacency-matrix factorisation
with PPR enhancement, as hand-written HIP kernels behind a C ABI
(include/damf.h).  This package is the thin Python binding."""
from ._damf import (  # noqa: F401
    Context,
    DamfConfig,
    DamfError,
    DAMF_DEVICE_PTRS,
    LIB_PATH,
    Server,
    default_config,
    lib,
    server_config,
)
