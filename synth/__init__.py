"""Seeded synthetic DNA read sets shared by the oracle tests, the GPU tests and
the benchmark.

This package only simulates sequencing (genomes, read sampling, strand,
substitutions, indels, 'N' calls).  It holds none of the k-mer counting
arithmetic: no k-mer extraction, encoding, hashing or filter logic.
"""
from .reads import (  # noqa: F401
    ReadSet,
    concat_reads,
    config,
    config_names,
    random_reads,
    reads_from_strings,
)
from .serving import Request, ServingWorkload, sample_reads_fast, serving_workload  # noqa: F401
