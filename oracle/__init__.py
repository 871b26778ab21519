"""CPU oracle for sPEGG's per-generation update -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never does, and this package imports nothing from it.
"""
from .oracle import (  # noqa: F401
    OracleEcology,
    OracleParams,
    OraclePop,
    OracleStats,
    binomial_thresholds,
    find_gap_word,
    geometric_thresholds,
    load,
    normals,
    philox4x32_10,
    poisson_thresholds,
    prob_threshold,
    recomb_mode,
    skip_gap,
    small_binomial_thresholds,
)
