"""Seeded synthetic inputs for the overlapping-domain-decomposition ptychography path.

This package only draws inputs: complex test images, probes, raster scan offsets,
the frame-to-subdomain block partition and Poisson counts.  It contains none of
the reconstruction method's arithmetic (no Fourier transform, no proximal map, no
ADMM step): measured intensities are produced by whichever forward operator the
caller trusts and then handed to :func:`poisson_counts`.

Both the FP64 test oracle and the GPU library's tests/bench draw their inputs
from here, so the two sides always start from identical numbers.
"""
from .problems import (  # noqa: F401
    CONFIGS,
    ProblemSpec,
    smooth_field,
    make_image,
    make_probe,
    raster_positions,
    raster_offsets,
    block_partition,
    poisson_counts,
    draw_problem,
    batch_specs,
    crop_spec,
)
