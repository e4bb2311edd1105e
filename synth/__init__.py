"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This package only draws data (patterns X, targets t, workload shapes).  It holds
none of the fitness or genetic-operator arithmetic: the HIP path and the CPU
oracle each implement those on their own.
"""
from .generators import (  # noqa: F401
    DATA_SEED_BASE,
    data_seed,
    ga_seed,
    regression_dataset,
    classification_dataset,
    batched_workload,
    random_population,
    random_fitness,
    sha256_arrays,
)
