"""Seeded synthetic inputs shared by the tests, the oracle checks and the bench.

Holds no KDE arithmetic; see ais.py."""
from .ais import (BOX_C1, BOX_C2, Box, MapSpec, Tracks, batch_specs, compression_ratio, dp_compress, generate, mercator,
                  metres_per_degree, window_tracks, workload_lanes, workload_small)

__all__ = ["BOX_C1", "BOX_C2", "Box", "MapSpec", "Tracks", "batch_specs", "compression_ratio", "dp_compress", "generate", "mercator",
           "metres_per_degree", "window_tracks", "workload_lanes", "workload_small"]
