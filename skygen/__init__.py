"""Seeded synthetic sky generator shared by the tests, the smoke check and the benchmark.

The generator only draws inputs (bands, noise levels, positions, spectral-parameter fields,
amplitudes, noise, spherical K-means labels, latitude masks, parameter points).  It contains no
part of the likelihood or of the mixing-matrix code used by either the oracle or the HIP library.
"""

from .sky import (  # noqa: F401
    BOUNDS,
    X0,
    ScanTasks,
    Sky,
    bands,
    kcap_labels,
    latitude_mask,
    make_config,
    make_tiny,
    scan_tasks,
    sky_sed_dust,
    sky_sed_sync,
    spherical_kmeans,
    start_and_box,
)
