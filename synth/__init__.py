"""Seeded synthetic workloads shared by the oracle tests, the device tests and
the benchmark.  This package holds input generation only: none of the matching
arithmetic lives here."""
from .common import MASTER_SEED, scale_tables, level_allocation  # noqa: F401
from .configs import (config, config1, config2, config3, config4,  # noqa: F401
                      seed_of, tiny_clustered, tiny_fisheye, tiny_pinhole)
