"""Seeded synthetic point-cloud pairs (inputs only; no registration arithmetic).

Both the FP64 oracle tests and the GPU path draw their inputs from here, so
this package holds scene synthesis, sampling, ray casting and ground-truth
poses only.  Nothing in it builds a mixture tree or registers a cloud.
"""

from .scenes import (  # noqa: F401
    PairSample,
    BatchSample,
    small_pair,
    lidar_pair,
    lidar_sequence,
    SequenceSample,
    depth_pair,
    uneven_batch,
    rotation_from_axis_angle,
    rotation_angle_deg,
    blob_tree_cloud,
    as_soa,
)
