"""Seeded synthetic inputs (road graphs, vehicles) shared by tests, benchmarks
and the oracle.  Holds no routing arithmetic."""
from .roadgraph import (RoadGraph, Vehicles, Workload, grid_graph, planar_graph, pack_graphs,
                        random_od, shell_od, default_params, grid8, grid32, planar100k, multi_city,
                        from_edges, serving_city, query_stream)
