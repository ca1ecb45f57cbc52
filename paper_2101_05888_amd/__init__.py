"""MI355X-native time-domain backprojection for synthetic aperture sonar.

The computation lives in the HIP library ``libsas_bp.so`` (C ABI in
``include/sas_bp.h``); this package is its binding. Any call into it without
the built library raises ``ImportError``: there is no CPU fallback.
"""
from .api import (Plan, SwathBuffers, swath_desc, sas_bp_plan, sas_bp_workspace_size, sas_bp_image,
                  sas_bp_adjoint, sas_bp_reproject, sas_bp_drc, sas_bp_tvg, sas_bp_envelope, sas_bp_whiten, sas_bp_range_compress, sas_bp_dpc_tde, dpc_desc, sas_bp_dpc_footprints, sas_bp_dpc_residual, sas_bp_dpc_fine_delay, sas_bp_dpc_solve, sas_bp_useful_updates, sas_bp_sharpness, sas_bp_sharpness_static, sas_bp_autotune, sas_bp_gate_class, sas_bp_set_kernel_timing,
                  sas_bp_kernel_time, sas_bp_abi_version)
from ._native import SasBpError

__all__ = ["Plan", "SwathBuffers", "swath_desc", "sas_bp_plan", "sas_bp_workspace_size", "sas_bp_image",
           "sas_bp_adjoint", "sas_bp_reproject", "sas_bp_drc", "sas_bp_tvg", "sas_bp_envelope", "sas_bp_whiten", "sas_bp_range_compress", "sas_bp_dpc_tde", "dpc_desc", "sas_bp_dpc_footprints", "sas_bp_dpc_residual", "sas_bp_dpc_fine_delay", "sas_bp_dpc_solve", "sas_bp_useful_updates", "sas_bp_sharpness", "sas_bp_sharpness_static", "sas_bp_autotune", "sas_bp_gate_class", "sas_bp_set_kernel_timing",
           "sas_bp_kernel_time", "sas_bp_abi_version", "SasBpError"]
