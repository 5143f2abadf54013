"""Seeded synthetic graph generators shared by the tests, the oracle checks and
the benchmark.  This package holds no arithmetic of the coarsening method:
it only builds input graphs (symmetric CSR with integer weights)."""
from .graphs import (CSR, csr_from_edges, grid2d, rgg, rmat, random_graph,  # noqa: F401
                     path_graph, cycle_graph, star_graph, complete_graph, batch_graphs,
                     degrade_grid, serve_requests, rgg_points)
