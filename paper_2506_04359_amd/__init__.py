"""MI355X (gfx950) sliding-window sparse Levenberg-Marquardt bundle adjustment.

Thin Python binding of ``libba.so`` (C ABI in ``include/ba.h``).  Every step of
the solve runs in the library's HIP kernels; this module only marshals
arguments: host index lists for plan creation, torch tensors for device memory
and the caller's current HIP stream.  Loading fails loudly when the library has
not been built (``python -m paper_2506_04359_amd.build``); there is no fallback.
"""
from ._binding import (  # noqa: F401
    BA_CREATE_HOST_ONLY,
    BA_ERR_HIP,
    BA_ERR_INVALID_ARG,
    BA_ERR_OOM,
    BA_ERR_STATE,
    BA_ERR_UNSUPPORTED,
    BA_ERR_WORKSPACE_TOO_SMALL,
    BA_FP64,
    BA_MIXED,
    BA_OK,
    BAError,
    Batch,
    Rig,
    Settings,
    REPORT_DTYPE,
    VI_PREINT_DOUBLES,
    Window,
    adjoint,
    lib,
    parse_reports,
    parse_traces,
    pnp_solve,
    triangulate,
    Graph,
    Map,
    pgo_solve,
    solve,
    solve_batched,
    solve_noalloc,
    vi_preintegrate,
    vi_solve,
    vi_workspace_size,
)
from .autograd import BASolve  # noqa: F401
