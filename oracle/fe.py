"""ORACLE (test infrastructure only): finite element basis, geometry and
assembly.

Paper Sec. 2 discretises the Kohn-Sham problem with linear Lagrange elements
on a tetrahedral decomposition; the stiffness and potential-weighted mass
matrices of Sec. 3.3 (eqs. st3, st4) are the integrals assembled here.
Reading: P1 as in the paper, plus P2 Lagrange on affine tetrahedra (edge
nodes at straight midpoints) for the larger workloads; all integrals use the
supplied quadrature rule, which defines where potentials are sampled.
"""
import numpy as np
import scipy.sparse as sp

P2_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def basis_tables(order, bary):
    """Values phi[q][a] and barycentric derivatives dphi[q][a][v] =
    d phi_a / d lambda_v of the Lagrange basis at the quadrature points.

    P1: phi_a = lambda_a.
    P2: phi_a = lambda_a (2 lambda_a - 1) at vertices, 4 lambda_a lambda_b on
    the edges 01, 02, 03, 12, 13, 23."""
    lam = np.asarray(bary, dtype=np.float64)
    nq = lam.shape[0]
    if order == 1:
        phi = lam.copy()
        dphi = np.zeros((nq, 4, 4))
        for a in range(4):
            dphi[:, a, a] = 1.0
        return phi, dphi
    phi = np.zeros((nq, 10))
    dphi = np.zeros((nq, 10, 4))
    for a in range(4):
        phi[:, a] = lam[:, a] * (2.0 * lam[:, a] - 1.0)
        dphi[:, a, a] = 4.0 * lam[:, a] - 1.0
    for e, (a, b) in enumerate(P2_EDGES):
        phi[:, 4 + e] = 4.0 * lam[:, a] * lam[:, b]
        dphi[:, 4 + e, a] = 4.0 * lam[:, b]
        dphi[:, 4 + e, b] = 4.0 * lam[:, a]
    return phi, dphi


def element_geometry(coords, elems):
    """Affine map x = X0 + J xi of every element.  Returns J [n_e][3][3]
    (columns X1-X0, X2-X0, X3-X0), det J, and the barycentric gradients
    grad_lambda [n_e][4][3] (rows of J^{-1}; grad lambda_0 = -sum of the
    others).  Raises on a non-positive determinant (inverted element)."""
    X = coords[elems[:, :4]]                      # [n_e][4][3]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    det = np.linalg.det(J)
    if np.any(det <= 0.0):
        raise ValueError("mesh has an element with det J <= 0")
    Jinv = np.linalg.inv(J)                       # row v-1 = grad lambda_v
    gl = np.empty((elems.shape[0], 4, 3))
    gl[:, 1:4, :] = Jinv
    gl[:, 0, :] = -Jinv.sum(axis=1)
    return J, det, gl


def quad_points(coords, elems, bary):
    """Physical quadrature points x_eq = sum_v lambda_v(q) X_v  [n_e][n_q][3]."""
    X = coords[elems[:, :4]]
    return np.einsum("qv,evd->eqd", bary, X)


def quad_weights(det, w):
    """dV_eq = w_q |det J_e|: the discrete measure of every quadrature point."""
    return det[:, None] * w[None, :]


def element_matrices(order, quad, det, gl, V=None, kind="mass"):
    """Element matrices by quadrature.
      stiffness:  K_e[a][b] = sum_q dV_q grad phi_a . grad phi_b
      mass:       M_e[a][b] = sum_q dV_q phi_a phi_b
      potential:  M_e[V][a][b] = sum_q dV_q V_q phi_a phi_b"""
    phi, dphi = basis_tables(order, quad.bary)
    dV = quad_weights(det, quad.w)                # [n_e][n_q]
    if kind == "stiffness":
        # grad phi_a at q = sum_v dphi[q,a,v] grad lambda_v
        g = np.einsum("qav,evd->eqad", dphi, gl)
        return np.einsum("eq,eqad,eqbd->eab", dV, g, g)
    if kind == "mass":
        return np.einsum("eq,qa,qb->eab", dV, phi, phi)
    if kind == "potential":
        return np.einsum("eq,qa,qb->eab", dV * V, phi, phi)
    raise ValueError(kind)


def assemble(n_nodes, elems, Ae):
    """Global matrix over all nodes: the sum over elements of the element
    matrices placed at their node ids (duplicates summed)."""
    nl = elems.shape[1]
    rows = np.repeat(elems, nl, axis=1).ravel()
    cols = np.tile(elems, (1, nl)).ravel()
    A = sp.coo_matrix((Ae.ravel(), (rows, cols)), shape=(n_nodes, n_nodes)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def restrict(A, rows, cols):
    """Sub-matrix A[rows][:, cols] (CSR)."""
    return A[rows][:, cols].tocsr()


def eval_at_quad(order, quad, elems, U):
    """u(x_eq) = sum_a phi_a(q) U[node_a] for nodal values U [n_nodes] or
    [n_nodes][k]."""
    phi, _ = basis_tables(order, quad.bary)
    Ue = U[elems]                                  # [n_e][n_loc](...)
    if U.ndim == 1:
        return np.einsum("qa,ea->eq", phi, Ue)
    return np.einsum("qa,eak->eqk", phi, Ue)


def density_at_quad(order, quad, elems, psi_nodes, occ):
    """rho(x_q) = sum_i f_i psi_i(x_q)^2 (Sec. 2 with occupations f_i; the
    examples of Sec. 4 use f_i = 2)."""
    pq = eval_at_quad(order, quad, elems, psi_nodes)
    return np.einsum("eqk,k->eq", pq * pq, np.asarray(occ, dtype=np.float64))


def load_vector(order, quad, elems, det, n_nodes, f_q):
    """b_a = sum_e sum_q dV_eq f_q phi_a(x_q) over all nodes."""
    phi, _ = basis_tables(order, quad.bary)
    dV = quad_weights(det, quad.w)
    be = np.einsum("eq,qa->ea", dV * f_q, phi)
    return np.bincount(elems.ravel(), weights=be.ravel(), minlength=n_nodes)
