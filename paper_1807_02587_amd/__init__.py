"""GMM-Tree point cloud registration on MI355X (gfx950).

Thin Python binding over the C ABI of ``libhgmm.so`` (see include/hgmm.h).
PyTorch provides device memory and streams; every step of construction and
registration runs in the library's HIP kernels.
"""

from ._lib import HgmmError  # noqa: F401
from .api import (  # noqa: F401
    Tree,
    Workspace,
    hgmm_build,
    hgmm_register_flat,
    hgmm_point_loglik,
    hgmm_register_soft,
    hgmm_estep_soft,
    hgmm_odometry,
    hgmm_estep_flat,
    hgmm_register,
    hgmm_register_noalloc,
    hgmm_build_batch,
    hgmm_register_batch,
    hgmm_register_warm_batch,
    hgmm_estep_batch,
    MLP,
    hgmm_warm_features,
    hgmm_warm_head_pose,
    hgmm_warm_head_target,
    hgmm_gemm_bf16,
    hgmm_estep,
    hgmm_normal_equations,
    hgmm_tree_import,
    hgmm_tree_nodes,
    hgmm_level_offset,
    hgmm_set_tuning,
    hgmm_get_tuning,
    hgmm_autotune,
    TUNING_KEYS,
    library_path,
    hgmm_profile,
    hgmm_profile_reset,
    hgmm_profile_read,
    PROFILE_KINDS,
)
