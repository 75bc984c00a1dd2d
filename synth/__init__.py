"""Seeded synthetic inputs for the BSGD-TV reconstruction problem.

This package generates problem instances only: the projection matrix A of a
2-D parallel-beam geometry (exact ray-pixel chord lengths), seeded
random-ellipse phantoms x_true, and noisy projections y = A x_true + noise.
It holds none of the reconstruction method's arithmetic.  Both the FP64
oracle (``oracle/``) and the device path take its output as input; neither
of them is imported here.
"""
from .problem import (  # noqa: F401
    CONFIGS,
    Problem,
    block_offsets,
    block_subsets,
    build_native,
    ellipse_phantom,
    make_problem,
    make_volume_problem,
    projection_matrix,
    seeded_vector,
    transpose_csr,
)
