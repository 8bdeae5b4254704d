"""Seeded synthetic sparse-matrix inputs.

This package only *builds inputs*: CSR patterns, values and dense vectors
drawn from ``numpy.random.Generator(PCG64(seed))``.  It contains none of the
arithmetic of the sparse matrix-vector method itself, so that both the CPU
oracle and the HIP library can consume the same bytes without sharing any
computation.
"""
from .generators import (  # noqa: F401
    CSR,
    zipf_degrees,
    gen_uniform_zipf,
    gen_c1,
    gen_c2,
    gen_c3_spd,
    gen_c4_batch,
    gen_c4_one,
    gen_family,
    gen_vectors,
    gen_block_hidden,
    gen_banded_like,
    gen_locality,
    LOCALITY_KINDS,
    csr_sha256,
)
