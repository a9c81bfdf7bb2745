"""libkfpswr: Schwarz waveform relaxation for the Kolmogorov equation on MI355X.

Thin Python binding over the C ABI of ``include/kfpswr.h``.  Every step of the
method runs in the library's HIP kernels; this module only marshals torch
tensors (device memory) and the current HIP stream into the C calls.  The
shared library must have been built (``python -m paper_1306_4596_amd.build``);
a missing library raises, there is no other code path.
"""
from __future__ import annotations

from .binding import (  # noqa: F401
    DIRICHLET,
    MLP,
    PARALLEL,
    RED_BLACK,
    FD,
    FEM,
    ROBIN,
    KfpError,
    SWRStats,
    axpy_f32,
    bw_probe,
    tile_probe,
    cast_f64_f32,
    column_stats,
    destandardize,
    trace_modes,
    trace_synth,
    get_config,
    get_batch_launch,
    get_launch,
    get_launch_tiles,
    lib_path,
    load_library,
    mono_solve,
    mono_solve_static,
    mul_f32,
    release_workspace,
    reload_tune_cache,
    set_config,
    set_kernel_timing,
    set_ordering,
    set_scheme,
    set_pipeline,
    standardize,
    subdomain_rows,
    swr_batch,
    swr_solve,
    swr_solve_windows,
    tune,
    tune_batch,
    u0_guess,
)
