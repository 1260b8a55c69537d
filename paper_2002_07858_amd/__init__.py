"""MI355X-native Feldman-Cousins grid scan (arXiv:2002.07858), HIP for gfx950.

The computation lives in libfc.so (C ABI in include/fc.h); this package is its
thin Python binding (``fc``) plus a convenience driver (``scan_problem``) that
runs the whole hot path on one grid and returns device tensors.
"""
from .fc import (FC_ERR_DEVICE, FC_ERR_INVALID_ARG, FC_ERR_NOMEM, FC_ERR_NOT_PD,
                 FC_ERR_STATE, FC_ERR_UNSUPPORTED, FC_FORM_FP32, FC_FORM_FP64,
                 FC_FORM_SPLIT_BF16, FC_FORM_SPLIT_FP16, FC_MAX_BINS, FC_NO_ALLOC_SCRATCH_BYTES, FC_OK, FC_STAT_FIXED,
                 FC_REQ_DONE, FC_REQ_FAILED, FC_REQ_QUEUED, FC_REQ_RUNNING, FC_SCHED_FAIR,
                 FC_SCHED_FIFO,
                 FC_STAT_PEARSON, FCError, Grid, Server, fc_acceptance, fc_build_covariance,
                 fc_build_grid, fc_critical_value, fc_data_scan, fc_generate_universes, fc_region,
                 fc_scan_fixed_m, fc_grid_destroy, fc_grid_device_bytes, fc_grid_info,
                 fc_grid_inverse_cov, fc_last_error, fc_profile_enable, fc_profile_read,
                 fc_scan, fc_scan_no_alloc, fc_scan_points,
                 fc_scan_points_slice, fc_scan_points_slice_workspace, fc_scan_points_workspace,
                 fc_scan_slice, fc_scan_state_finalize, fc_scan_state_init, lib)
from .driver import ScanOutputs, scan_problem

__all__ = [n for n in dir() if n.startswith("fc_") or n.startswith("FC")] + [
    "Grid", "Server", "lib", "ScanOutputs", "scan_problem"]
