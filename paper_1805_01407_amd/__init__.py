"""slrng: bulk generation from the scrambled linear generators of Blackman &
Vigna ("Scrambled Linear Pseudorandom Number Generators") on MI355X.

The work is done by ``libslrng.so`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/slrng.h``).  This package is a thin ctypes binding with
the same function names; PyTorch only supplies device memory and streams.
Importing the package does not load the library; the first call does, and it
raises if the library has not been built (``python -m
paper_1805_01407_amd.build``).
"""
from .binding import (  # noqa: F401
    VARIANTS, VARIANTS32, VARIANT_IDS, SlrngError, Streams, lib, library_path,
    slrng_version, slrng_strerror, slrng_last_hip_error, slrng_state_words,
    slrng_charpoly, slrng_jump_poly, slrng_jump_poly_device,
    slrng_streams_create, slrng_streams_create_from_states, slrng_streams_count,
    slrng_streams_variant, slrng_streams_seed,
    slrng_streams_jump, slrng_streams_advance, slrng_streams_advance_each, slrng_generate, slrng_linear_complexity,
    slrng_equidistribution_rank, slrng_gf2_rank, equidistribution_rank, gf2_rank,
    slrng_get_state, slrng_set_state, slrng_streams_destroy,
    slrng_get_tuning, slrng_set_tuning, slrng_calib_write, slrng_calib_copy,
    slrng_output_alloc, slrng_output_free, output_empty,
    SLRNG_U64, SLRNG_F64, SLRNG_U32, SLRNG_F32, SLRNG_JUMP, SLRNG_LONG_JUMP,
    SLRNG_BATCH_GRAPH, SLRNG_BATCH_PERSISTENT, SLRNG_BATCH_PLAIN, SLRNG_BATCH_STATIC_SCRATCH_BYTES,
    REQUEST_DTYPE, make_requests,
    slrng_batch_default_opts, slrng_batch_plan, slrng_batch_launch, slrng_batch_info,
    slrng_batch_destroy, slrng_batch_run, slrng_batch_run_static, slrng_batch_latencies,
    set_batch_defaults,
    SLRNG_SUBMIT_NONBLOCK, SLRNG_SUBMIT_AUTORELEASE, slrng_server_default_opts,
    slrng_server_create, slrng_server_submit, slrng_server_poll, slrng_server_wait,
    slrng_server_release, slrng_server_drain, slrng_server_get_stats, slrng_server_reset_stats,
    slrng_server_replay, slrng_server_destroy, slrng_server_advance, slrng_server_intervals,
)
