"""MI355X-native non-linear digital tracking (HIP / gfx950).

Thin Python binding of ``libdtrack.so`` (declared in ``include/dtrack.h``).
It marshals arguments only: every step of the tracking path runs in the
library's HIP kernels.  PyTorch supplies device memory and the stream.
There is no fallback: if the library is missing, importing the binding's
functions raises.
"""
from .binding import (  # noqa: F401
    DtrackError, Context, Patch, OrbitSet, lib, stack, topk, debug_samples, validate_orbits,
    exposure_struct, LIB_PATH, stack_batched, autotune_batched, batch_outputs, cell_stamps, stack_cells,
    gemm_bf16, Scorer, clip_candidates, image_noise, record_valid_gathers, replay_valid_gathers, GatherRecord,
    orbit_sampler, generate_orbits,
    stack_generated, topk_noalloc, cell_members_near, stack_ids, segment_max,
)
