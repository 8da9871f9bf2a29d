"""Exact contraction of planar square-lattice tensor networks on MI355X.

A thin ctypes binding over ``libtn.so`` (the C ABI in ``include/tn.h``): it
only marshals arguments.  Every step of a contraction runs in the library's
HIP kernels; PyTorch supplies device memory and the stream.  Importing this
package fails loudly if the library has not been built
(``python paper_1908_08553_amd/build.py``).
"""
from ._native import (  # noqa: F401
    TN_OK, TN_PENDING, TN_EINVAL, TN_ENOMEM, TN_EBUSY, TN_EDEVICE, TN_ENOTFOUND,
    TN_ENONFINITE, TN_EOVERFLOW,
    TN_ORDER_COLSWEEP, TN_ORDER_QUADRANT, TN_ORDER_HEURISTIC, TN_ORDER_SWEEP_AUTO,
    TN_ORDER_ROWS, TN_ORDER_ROWS_T,
    TN_PREC_F64, TN_PREC_F32, TN_PREC_BF16X3,
    TnError, Plan, Result, lib, library_path,
    tn_plan_grid, tn_plan_stats, tn_plan_text, tn_contract_grid, tn_set_option,
    tn_contract_grid_static, TN_STATIC_SCRATCH_BYTES,
    TN_OPT_KERNEL_IMPL, TN_OPT_BATCH_THREADS, TN_OPT_FUSE_STEPS, TN_OPT_CHUNK_SCHEDULE,
    TN_OPT_QUADRANT_STREAMS, TN_OPT_CHAIN_STEPS, TN_OPT_ENV_STREAMS, TN_OPT_ENV_ROWS,
    TN_OPT_ENV_SITES, TN_OPT_RING_OPERAND_SCALE, TN_OPT_CHUNK_STREAM,
    tn_profile_enable, tn_profile_read,
    Batch, tn_batch_workspace, tn_contract_batch, Server, EnvSet, Ite,
    plan_grid, contract_grid, device_sites, workspace_for,
    tn_double_layer, tn_double_layer_prepare, tn_observables, Sites, prepare_sites,
)
