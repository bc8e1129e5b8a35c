"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.  This module holds none of the method's arithmetic: it only lists
(alpha, n, replicates, seed, stream) cells and draws request datasets with
numpy's own generators."""
from .workloads import (TABLE_ALPHAS, TABLE_NS, heavy_tail, serving_requests,  # noqa: F401
                        single_cell, table_cells, table_slice, uneven_cells)
