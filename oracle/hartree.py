"""ORACLE (test infrastructure only): Hartree potential, Sec. 3.1.

The Hartree potential solves -Laplace V_H = 4 pi rho in the box with the
multipole boundary data w_D of eq. (bd): monopole Q/|d|, dipole p.d/|d|^3
and quadrupole, about the charge centre x'' = <x rho> / <rho>, d = x - x''.

Reading of the quadrupole factor: with raw second moments
q_ij = int rho (x_i - x''_i)(x_j - x''_j), the Taylor expansion of 1/|x-x'|
gives (1/2) sum q_ij (3 d_i d_j - delta_ij |d|^2) / |d|^5; the paper prints
no 1/2, kept as the option ``quad_factor=1``.  The dipole p vanishes about
the charge centre but is computed anyway.

The Galerkin problem on interior nodes I with boundary nodes B fixed to w_D,
    K_II V_I = 4 pi b_I - K_IB w_B,   b_a = <rho, phi_a>
(K the stiffness matrix without the 1/2 of the kinetic term), is solved by
KSProblem.hartree_nodes in step.py.
"""
import numpy as np


def density_moments(rho_q, x_q, dV):
    """Q = <rho, 1>, centre x'', dipole p_i and raw second moments q_ij."""
    Q = float(np.sum(dV * rho_q))
    c = np.einsum("eq,eqd->d", dV * rho_q, x_q) / Q
    d = x_q - c[None, None, :]
    p = np.einsum("eq,eqd->d", dV * rho_q, d)
    q = np.einsum("eq,eqi,eqj->ij", dV * rho_q, d, d)
    return Q, c, p, q


def multipole_boundary(points, Q, c, p, q, quad_factor=0.5):
    """w_D at the given points (eq. bd)."""
    d = points - c[None, :]
    r2 = np.sum(d * d, axis=1)
    r = np.sqrt(r2)
    mono = Q / r
    dip = (d @ p) / (r2 * r)
    quad = (3.0 * np.einsum("ni,ij,nj->n", d, q, d) - np.trace(q) * r2) / (r2 * r2 * r)
    return mono + dip + quad_factor * quad
