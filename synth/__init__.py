"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package draws pattern sets, texts and planted pattern copies from numpy's
Mersenne Twister (the paper draws its patterns with MT19937, Results section).
It holds none of the matching arithmetic: it never decides where a pattern
occurs, it only writes bytes and records where it wrote copies.
"""

from .workloads import (  # noqa: F401
    SEED_BASE,
    PatternSet,
    Workload,
    make_patterns,
    make_text,
    plant,
    c1_plain_small,
    c2_signature_set,
    c3_dna,
    c4_batched,
    c5_requests,
    workload,
)
