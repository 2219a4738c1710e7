"""SAFR per-frame atmospheric tomography on AMD Instinct MI355X (gfx950).

The reconstruction runs in the HIP library ``libsafr.so`` (C ABI in
``include/safr.h``); ``safr`` is its thin Python binding.
"""
from . import safr  # noqa: F401
from .safr import (Plan, SafrError, precompute_geometry, reconstruct, safr_destroy,  # noqa: F401
                   safr_export_B, safr_plan_info, safr_precompute, safr_reconstruct,
                   safr_reconstruct_batched, safr_set_option, safr_set_workspace, safr_workspace_size)
