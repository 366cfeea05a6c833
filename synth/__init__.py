"""Seeded synthetic inputs for the Euclidean-median workloads.

This package only draws data: images, noise and point sets with the shapes,
sizes and value distributions of the paper's experiments (Section 3: grey
images, additive Gaussian noise of level sigma, search window S = 21, patch
side k = 7, h = 10 sigma) and of the batched point-set workload.  It holds none
of the method's arithmetic (no patches, no weights, no ADMM), so both the FP64
oracle and the GPU path can consume its output without sharing code.
"""

from .images import (  # noqa: F401
    gradient_shapes_image,
    piecewise_smooth_image,
    add_gaussian_noise,
    add_impulses,
    psnr,
)
from .pointsets import PointSetBatch, make_pointset_batch  # noqa: F401
from .configs import (  # noqa: F401
    NlemWorkload,
    nlem_small,
    nlem_256,
    nlem_512_mixed,
    nlem_multi_image,
    pointset_workload,
    study_images,
    study_noise,
    STUDY_SIGMAS,
)
