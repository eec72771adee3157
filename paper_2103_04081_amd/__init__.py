"""MI355X-native block-randomized SGD with importance sampling for CP decomposition.

The compute lives in ``libcpdmi.so`` (HIP kernels for gfx950 behind the C ABI
of ``include/cpd.h``); :mod:`paper_2103_04081_amd.cpdmi` is its ctypes
binding.  Build with ``python -m paper_2103_04081_amd.build``.
"""

from .cpdmi import (  # noqa: F401
    Batch, CpdError, Decomposition, Server, cpd_poll, cpd_server_create, cpd_server_destroy,
    cpd_server_stats, cpd_submit, cpd_batch_create, cpd_batch_destroy, cpd_batch_fits,
    cpd_batch_member_info, cpd_batch_read_factors, cpd_batch_run, cpd_batch_step, cpd_batch_sync,
    cpd_batch_workspace_size, cpd_destroy, cpd_fit, cpd_get_step, cpd_init, cpd_read_cdf,
    cpd_read_factors, cpd_read_state, cpd_sample, cpd_step, cpd_step_replay, cpd_sync, cpd_variance,
    cpd_workspace_size, cpd_write_state, lib, make_options, make_problem)
