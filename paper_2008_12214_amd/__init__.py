"""MI355X-native hologram generation (HoloGen's iterative Fourier transform hot path).

The compute path is the HIP library ``libhologen.so`` (C ABI in
``include/hologen.h`` and ``include/hologen_nn.h``).  This package is a thin ctypes binding with the same
entry-point names: it checks tensor placement, allocates outputs and the
workspace through PyTorch, and passes raw device pointers and the current
stream.  Every step of the path runs in the library's kernels; there is no
CPU fallback, and importing fails loudly if the library has not been built.
"""
from ._binding import (  # noqa: F401
    HG_OK, HG_ERR_INVALID_ARG, HG_ERR_UNSUPPORTED_SIZE, HG_ERR_WORKSPACE, HG_ERR_HIP, HG_ERR_NUMERIC,
    HG_OP_GS, HG_OP_WGS, HG_OP_OSPR, HG_OP_PROPAGATE,
    HologenError, lib, lib_path,
    hg_workspace_size, hg_gs, hg_wgs, hg_wgs_static, HG_STATIC_SCRATCH_BYTES, HG_SLM_AMPLITUDE, HG_FIELD_FP16, hg_search, hg_search_workspace_size, HG_SEARCH_DS, HG_SEARCH_SA, hg_gs_step, hg_numeric_status, hg_lt, hg_ospr, hg_ospr_batched, hg_fresnel_propagate,
    hg_gs_batched, hg_gs_batched_workspace_size, hg_random_phase, hg_status_string, hg_last_error,
    hg_timing_enable, hg_timing_read, hg_autotune, hg_set_launch_config, hg_get_launch_config,
    hg_set_small_fused, hg_set_column_kernel, hg_set_batch_chunk, hg_get_batch_chunk, COLUMN_TILE, COLUMN_PERSISTENT, COLUMN_CLASSIC,
    hg_nn_param_count, hg_nn_workspace_size, hg_nn_workspace, hg_nn_forward, hg_nn_backward, hg_nn_adam,
    hg_replay_phase_init, hg_quadratic_phase_apply, hg_nn_pack_weights, hg_nn_conv3x3, hg_nn_conv3x3_wgrad, hg_nn_avgpool2,
    hg_nn_avgpool2_backward, hg_nn_upsample_concat, hg_nn_upsample_concat_backward, hg_nn_head,
    hg_nn_head_backward, hg_nn_phase_loss,
)
