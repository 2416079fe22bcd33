"""MI355X (gfx950) implementation of the per-mesh step of the nonnested
augmented subspace method for the Kohn-Sham equation (arXiv 2404.19249).

The computation lives in the HIP library ``_lib/libks.so`` behind the C ABI
of ``include/ks.h``; this package only marshals arguments.
"""
from .binding import load_library, KSError, header_functions, LIB_PATH
from .context import KSContext, KSBatch, stream_probe, mesh_metric, move_nodes, interpolate_field

__all__ = ["load_library", "KSError", "header_functions", "LIB_PATH", "KSContext", "KSBatch", "stream_probe", "mesh_metric",
           "move_nodes", "interpolate_field"]
