"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package only *produces data*: structured tetrahedral meshes (P1 / P2),
a smooth seeded node-moving map, sampled nuclei, and the conical-product
quadrature table that defines where potentials and densities live.  It holds
none of the method's arithmetic (no basis functions, no assembly, no solves).

Workloads are shaped like the molecules of the paper's experiments (Sec. 4):
a box around a handful of nuclei, tetrahedral meshes refined near the nuclei,
1 to 40 doubly occupied orbitals.
"""
from .mesh import Mesh, freudenthal_mesh, move_nodes_toward_nuclei, jittered_coarse_mesh
from .quadrature import conical_rule, QuadRule
from .atoms import Atoms, sample_atoms
from .workloads import Workload, make_workload, WORKLOADS

__all__ = [
    "Mesh", "freudenthal_mesh", "move_nodes_toward_nuclei", "jittered_coarse_mesh",
    "conical_rule", "QuadRule", "Atoms", "sample_atoms",
    "Workload", "make_workload", "WORKLOADS",
]
