"""Method parameters of the benchmark workloads.

The paper fixes lambda_c = 0.01 (Sec. 4.1) and J = 8; it leaves the tree
construction to its reference [33], so the covariance floor reg_eps and the
minimum soft mass of a live child are this library's choices.  reg_eps is set
per workload: 1e-6 for the unit-cube scenes (noise 5e-3), 4e-3 m^2 for the
spinning scanner (about the squared spacing of neighbouring rings at 10 m; a
floor at the 2 cm range noise leaves ring-segment leaves so thin that the
registration diverges), 1e-3 m^2 for the depth camera: the smallest of 1e-5,
1e-4, 1e-3 and 4e-3 m^2 at which a registration from the identity ends where
the one started at the ground truth ends, on each of eight generated room
pairs (finer floors leave thin wall patches whose likelihood is so peaked
that some pairs diverge from the identity).
"""

PRESETS = {
    # planes + spheres in the unit cube, 10k points, 2 levels (64 leaves)
    "small": dict(levels=2, reg_eps=1e-6, min_mass=1.0, lambda_c=0.01),
    # 64-ring spinning scan, ~1.2e5 points, 4 levels (4096 leaves)
    "lidar": dict(levels=4, reg_eps=4e-3, min_mass=32.0, lambda_c=0.01),
    # 640x480 depth camera, ~2.9e5 points, 5 levels (32768 leaves)
    "depth": dict(levels=5, reg_eps=1e-3, min_mass=8.0, lambda_c=0.01),
}
