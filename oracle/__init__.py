"""ORACLE: plain, slow, FP64 CPU implementation of one step of the augmented
subspace method for the Kohn-Sham equation (arXiv 2404.19249).

This package is TEST INFRASTRUCTURE.  Only the test-suite, the smoke check
and the benchmark's CPU-baseline leg may import it.  It shares no code with
the HIP library (no kernels, headers, helpers or tables); both sides only
read the same seeded inputs from ``ks_inputs``.

Every function follows a passage of the paper, cited in its docstring.  Where
the paper is silent or ambiguous the reading taken is stated where it is
used.  Library primitives used as single steps: scipy.sparse products and
COO->CSR summation (assembly is a sum over elements), numpy.linalg.eigh for
the small dense eigenproblems, numpy.linalg.solve for the Anderson normal
equations; element-level shape derivatives by complex-step differentiation
(numpy.linalg.det and inv on complex arrays).

Parity status: every function is pinned by a CPU test (quadrature exactness,
closed-form element matrices, global invariants, the hydrogen closed form,
Gaussian Poisson and multipole closed forms, XC derivative identities,
brute-force dense eigensolves on tiny meshes, the nested-mesh identity,
Anderson's least-squares property and finite differences for the adjoint,
for the reverse mode through the truncated PCG and for the derivative with
respect to the mesh vertices (Pulay terms; rigid-motion invariance too);
the Hessian metric and node mover by exact recovery of linear and quadratic
functions, the eigenvalue clamp, fixed points and energy descent),
except the nonlinear inner SCF's physical value, which is pinned only through
self-consistency properties ("parity unpinned" for its absolute energy).
"""
from .fe import (basis_tables, element_geometry, quad_points, assemble, restrict,
                 eval_at_quad, density_at_quad)
from .xc import lda_xc
from .hartree import density_moments, multipole_boundary
from .solvers import jacobi_pcg
from .coarse import coarse_interpolation
from .step import (KSProblem, ks_scf_step, initial_guess, block_solve, small_eig, anderson_mix,
                   step_backward)

__all__ = [
    "basis_tables", "element_geometry", "quad_points", "assemble", "restrict",
    "eval_at_quad", "density_at_quad", "lda_xc", "density_moments",
    "multipole_boundary", "jacobi_pcg",
    "coarse_interpolation", "KSProblem", "ks_scf_step", "initial_guess",
    "block_solve", "small_eig", "anderson_mix", "step_backward",
]
