"""GMACO-P routing hot path on AMD Instinct MI355X (gfx950).

The work runs in the HIP kernels of ``libgmacop.so`` behind the C ABI in
``include/gmacop.h``; ``paper_2010_14244_amd.gmacop`` is the ctypes binding.
"""
from .gmacop import (GmacopError, Graph, DeviceBatch, Server, gmacop_graph_create, gmacop_route_batch, gmacop_stats_get,
                     gmacop_vehicle_tau_get,
                     gmacop_route_batch_device, gmacop_state_get, gmacop_release, library_path)

__all__ = ["GmacopError", "Graph", "DeviceBatch", "gmacop_graph_create", "gmacop_route_batch",
           "gmacop_route_batch_device", "gmacop_state_get", "gmacop_release", "library_path"]
