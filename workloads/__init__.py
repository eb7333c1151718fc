"""Seeded synthetic inputs for the population graph-coloring path.

This package builds graphs, vertex weights and the named workload shapes.
It holds none of the coloring method's arithmetic: no conflict counting,
no tabu search, no crossover and no scoring.  Both the CPU oracle and the
GPU path consume what it produces.
"""
from .graphs import (  # noqa: F401
    Graph,
    gnp,
    planted_partite,
    uniform_weights,
    dsatur_colors,
    is_valid_csr,
)
from .configs import WORKLOADS, workload  # noqa: F401
