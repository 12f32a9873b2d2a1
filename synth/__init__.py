"""Seeded synthetic inputs shared by the CPU oracle's tests and the GPU path.

This module only draws pixels: search images with natural-image statistics
(power spectrum falling as 1/f^beta), flat bright rectangles, thin line
segments and smooth saturated cloud blobs, and templates cut from an image
with optional contrast/brightness change and Gaussian noise.  It contains none
of the search method's arithmetic, so both sides of a parity test can take
their inputs from here without sharing any part of the computation.

The paper's satellite and aerial datasets (section VII) are not available;
these generators stand in for them.
"""

from .gen import (  # noqa: F401
    BASE_SEED,
    config_seed,
    spectral_image,
    add_rectangles,
    add_lines,
    add_clouds,
    aerial_image,
    cut_template,
    noise_template,
    workload,
    serving_queries,
    poisson_arrivals,
)
