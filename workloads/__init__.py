"""Seeded synthetic PSLG generators shared by the oracle tests and the GPU path.

This package holds input generation only: point sets, constraint segments and
the quality bound. It performs none of the refinement arithmetic.
"""
from .generators import (  # noqa: F401
    PSLG,
    bare_square,
    config0,
    config1,
    config2,
    scaled_config1,
    scaled_config2,
    spokes,
    near_edge_point,
    random_small,
    manifest_hash,
    BATCH_BOUNDS_SQ,
    batch_plan,
    batch_instance,
    batch_config3,
    serving_plan,
    serving_job,
    serving_jobs,
)
from .predicates import FAMILIES as PREDICATE_FAMILIES, predicate_corpus  # noqa: F401
