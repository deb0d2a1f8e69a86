"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package holds no arithmetic of the quantizer itself: it only draws images
and the random initial-center indices that the method takes as input (the
"random subset of the data" of the k-means initialisation, Sec. 2, Alg. 1 and
Alg. 2).  Both the CPU oracle and the GPU path receive exactly these arrays.
"""

from .images import (  # noqa: F401
    gradient_blob_image,
    sinusoid_field_image,
    workload_image,
    batched_workload,
    WORKLOADS,
)
from .palette import init_indices, unpack_keys_to_palette  # noqa: F401
