"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This package only draws random numbers; it holds none of the correlation
arithmetic, so neither the oracle nor the GPU path depends on the other
through it.
"""

from .workloads import (  # noqa: F401
    SEED_BASE,
    factor_matrix,
    cfg_plain_small,
    cfg_gpu_headline,
    cfg_precision,
    cfg_differentiation,
    cfg_serving_base,
    serving_queries,
    paper_shape,
    heavy_ties,
    edge_matrix,
    mode_selected,
    pvalue_matrix,
    categorical_continuous,
    categorical_matrix,
)
