"""Seeded synthetic case-control data sets for the three-way epistasis scan.

This package only draws inputs (genotype matrices, phenotype vectors,
phenotype permutations, uneven data-set batches).  It contains none of the
method's arithmetic (no tables, no scores) so that both the oracle and the
GPU library can consume the same inputs without sharing any code.
"""
from .generate import (  # noqa: F401
    CONFIGS,
    Dataset,
    SplitMix64,
    make_config,
    make_dataset,
    make_parity_fixture,
    make_permutations,
    make_uneven,
    manifest_sha256,
)
