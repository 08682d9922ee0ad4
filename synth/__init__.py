"""Seeded synthetic workloads shared by the oracle tests, the device tests and
the benchmark.  This package holds input generation only: none of the matching
arithmetic lives here."""
from .common import MASTER_SEED, scale_tables, level_allocation  # noqa: F401
from .motion import last_frame_case, motion_params  # noqa: F401
from .orb import orb_pattern  # noqa: F401
from .workloads import (SINGLE_FRAME, clustered_batch, clustered_search_20000, fisheye_frame_1500,  # noqa: F401
                        mixed_batch, pinhole_frame_1200, seed_of, tiny_clustered, tiny_fisheye,
                        tiny_pinhole, workload)
