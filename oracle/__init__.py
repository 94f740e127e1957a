"""CPU oracle for the deterministic MIS-2 and MIS-2 aggregation.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.
"""
from .oracle import (  # noqa: F401
    build_oracle,
    use_library,
    xorshift64star,
    hash_priority,
    id_bits,
    pack,
    mis2,
    mis2_ex,
    mis2_ablation,
    xorshift64,
    PRIO_FIXED,
    PRIO_XORSHIFT,
    aggregate,
    aggregate_basic,
    quotient,
    color_jp,
    cgs_plan,
    cgs_apply,
    galerkin,
    smoothed,
    coarsen,
)
