"""ORACLE (test infrastructure only): derivative of one step's Kohn-Sham
energy with respect to the vertex coordinates of the fine mesh, and nuclear
forces with mesh-motion (Pulay) terms.

The paper moves the mesh between steps (Algorithm 2, Sec. 3.2) but
differentiates nothing.  Reading: the map of one augmented-subspace step
(Algorithm 3) with its inputs held fixed -- the nodal coefficients of Psi^l,
lambda^l, rho^l at the quadrature points, the Hartree boundary data w_B and
the matrix of I_H^h (the coarse space is carried by the moving mesh) -- and
the vertices X of the fine mesh as the variables.  P2 edge nodes sit at
straight midpoints, so the geometry is that of the vertices.

With the inner iteration converged, Psi^{l+1} = Z U is stationary over
span(Z) for
    L = E_KS^step(Psi) - sum_i f_i theta_i (psi_i^T M psi_i - 1)
(the Sec. 2 functional with the step's frozen-boundary Hartree term), so
    dE/dX = dL/dX at fixed (Z, U)  +  < 2 R F U^T, dZ/dX >,
    R = A Psi - M Psi Theta (A: Hamiltonian of the final inner iteration),
with Z = [P | Psi_t], Psi_t = Psi_hat - P G^{-1} P^T M Psi_hat, G = P^T M P
and S Psi_hat = M Psi^l (Lambda^l + mu), S = 1/2 K + M[V_eff^l] + mu M.
Differentiating these relations one at a time:
  kinetic             1/2 sum_i f_i psi_i^T dK psi_i
  constraint          - sum_i f_i theta_i psi_i^T dM psi_i
  external, xc        sum_q d(dV_q) rho_q (V_ext + eps_xc) + sum_q dV_q rho_q dV_ext(x_q)
  Hartree, V_0 part   sum_q d(dV_q) rho_q V_0(q) - V_0^T dK V_0 / (8 pi)
  Hartree, V_bc part  sum_q d(dV_q) c_q V_bc(q) - W^T dK V_bc,
                      c = rho - rho^l / 2, K_II W = <c, phi_I>
  M-orthogonalisation - sum_i (P C)_i^T dM psi_t_i,  C = G^{-1} P^T Psi_bar_t
  BVP right side      sum_i (lambda_i + mu) Y_i^T dM psi^l_i,  S Y = Psi_bar_hat
  BVP operator        - sum_i Y_i^T (1/2 dK + mu dM) psi_hat_i
                      - sum_q d(dV_q) gamma_q V_eff^l(q) - sum_q dV_q gamma_q dV_ext(x_q)
                      - 4 pi sum_q d(dV_q) rho^l_q W2(q) + W2^T dK V_H^l,
                      gamma = sum_i Y_i psi_hat_i at q, K_II W2 = <gamma, phi_I>
where Psi_bar_t = 2 R F U_t^T and Psi_bar_hat = Psi_bar_t - M P C (the
adjoint of the step's implicit adjoint), V_0 = V_H[rho] with zero boundary
values, V_bc the discrete harmonic lift of w_B, V_H^l = V_H[rho^l] with w_B.
Every term is an element-level derivative of a stiffness form u^T K_e v, a
mass form u^T M_e v, sum_q dV_q F_q for fixed F_q, or sum_q dV_q G_q
V_ext(x_q) with moving points; this module takes those by complex-step
differentiation of the element quantities (exact to rounding, no step-size
error), one local vertex coordinate at a time.
"""
import numpy as np

from . import fe
from .xc import lda_xc
from .solvers import jacobi_pcg


def _element_forms(order, quad, Xe, kpairs, mpairs, F_q, G_q, Z, R):
    """Per element, for vertex coordinates Xe [n_e][4][3] (real or complex):
    sum over stiffness pairs of sum_i w_i u_i^T K_e v_i, the same over mass
    pairs with M_e, sum_q dV_q F_q, and sum_q dV_q G_q V_ext(x_q)."""
    phi, dphi = fe.basis_tables(order, quad.bary)
    J = np.stack([Xe[:, 1] - Xe[:, 0], Xe[:, 2] - Xe[:, 0], Xe[:, 3] - Xe[:, 0]], axis=2)
    det = np.linalg.det(J)                         # > 0 on a valid mesh
    Jinv = np.linalg.inv(J)                        # row v-1 = grad lambda_v
    gl = np.concatenate([-Jinv.sum(axis=1, keepdims=True), Jinv], axis=1)
    dV = det[:, None] * quad.w[None, :]
    out = np.einsum("eq,eq->e", dV, F_q)
    x = np.einsum("qv,evd->eqd", quad.bary, Xe)
    vext = np.zeros(x.shape[:2], dtype=x.dtype)
    for z, r in zip(Z, R):
        d = x - r[None, None, :]
        vext = vext - z / np.sqrt(np.sum(d * d, axis=-1))
    out = out + np.einsum("eq,eq,eq->e", dV, G_q, vext)
    g = np.einsum("qav,evd->eqad", dphi, gl)       # grad phi_a at q
    for ue, ve, w in kpairs:
        gu = np.einsum("eqad,eak->eqkd", g, ue)
        gv = np.einsum("eqad,eak->eqkd", g, ve)
        out = out + np.einsum("eq,eqkd,eqkd,k->e", dV, gu, gv, w)
    for ue, ve, w in mpairs:
        uq = np.einsum("qa,eak->eqk", phi, ue)
        vq = np.einsum("qa,eak->eqk", phi, ve)
        out = out + np.einsum("eq,eqk,eqk,k->e", dV, uq, vq, w)
    return out


def shape_derivative(prob, kpairs, mpairs, F_q, G_q, h=1e-30):
    """d/dX of the sum over elements of _element_forms at every node
    [n_nodes][3] (zero at P2 edge nodes).  Pairs are (U, V, w) with nodal
    arrays U, V [n_nodes][k] and column weights w [k]."""
    el = prob.elems
    gather = lambda A: A[el]                       # [n_e][n_loc][k]
    kp = [(gather(u), gather(v), np.asarray(w, dtype=np.float64)) for u, v, w in kpairs]
    mp = [(gather(u), gather(v), np.asarray(w, dtype=np.float64)) for u, v, w in mpairs]
    Xe = prob.coords[el[:, :4]]
    out = np.zeros((prob.n_nodes, 3))
    for v in range(4):
        for d in range(3):
            Xc = Xe.astype(np.complex128)
            Xc[:, v, d] += 1j * h
            val = _element_forms(prob.order, prob.quad, Xc, kp, mp, F_q, G_q, prob.Z, prob.R).imag / h
            np.add.at(out[:, d], el[:, v], val)
    return out


def step_mesh_gradient(prob, res, Psi_l, lam_l, tol=1e-14, tol_poisson=1e-14):
    """dE_KS(Psi^{l+1}) / dX at every node [n_nodes][3] for the step `res`
    from (Psi_l, lam_l) on `prob` (the module docstring lists the terms)."""
    k = res.Psi.shape[1]
    NH = prob.P.shape[1]
    Psi, U, th = res.Psi, res.U, np.asarray(res.lam, dtype=np.float64)
    occ = np.asarray(prob.occ, dtype=np.float64)
    lam_l = np.asarray(lam_l, dtype=np.float64)
    rho, rho_l, w_B = res.rho_q, res.extra["rho_l"], res.extra["w_B"]
    S, Z, G = res.extra["S"], res.extra["Z"], res.extra["G_PP"]
    nonlinear = prob.hartree or prob.xc_mode != "none"
    A = (prob.A_linear() + prob.potential_matrix(res.extra["vnl_in"])).tocsr() \
        if nonlinear else prob.A_linear()
    # dE/dZ on the Psi_t columns, then through the M-orthogonalisation
    R = A @ Psi - (prob.M_II @ Psi) * th[None, :]
    bar_t = 2.0 * (R * occ[None, :]) @ U[NH:NH + k, :].T
    PC = prob.P @ np.linalg.solve(G, prob.P.T @ bar_t)
    bar_h = bar_t - prob.M_II @ PC
    Y, _, _ = jacobi_pcg(S, bar_h, None, tol=tol, max_iter=200000)   # S symmetric
    Psi_t = Z[:, NH:NH + k]
    nodes = prob.to_nodes
    gam = np.einsum("eqk,eqk->eq", prob.at_quad(nodes(Y)), prob.at_quad(nodes(res.Psi_hat)))
    eps, _ = lda_xc(rho, prob.xc_mode)
    _, vxc_l = lda_xc(rho_l, prob.xc_mode)
    F = rho * eps - gam * vxc_l
    kpairs = [(nodes(Psi), nodes(Psi), 0.5 * occ),
              (nodes(Y), nodes(res.Psi_hat), -0.5 * np.ones(k))]
    if prob.hartree:
        zB = np.zeros_like(w_B)
        c = rho - 0.5 * rho_l
        VHl, _ = prob.hartree_nodes(rho_l, w_B, tol_poisson)
        Vbc, _ = prob.hartree_nodes(np.zeros_like(rho), w_B, tol_poisson)
        V0, _ = prob.hartree_nodes(rho, zB, tol_poisson)
        W, _ = prob.hartree_nodes(c / (4.0 * np.pi), zB, tol_poisson)       # K_II W = <c, phi>
        W2, _ = prob.hartree_nodes(gam / (4.0 * np.pi), zB, tol_poisson)    # K_II W2 = <gam, phi>
        q = prob.at_quad
        F = F + rho * q(V0) + c * q(Vbc) - gam * q(VHl) - 4.0 * np.pi * rho_l * q(W2)
        col = lambda v: v[:, None]
        kpairs += [(col(V0), col(V0), [-1.0 / (8.0 * np.pi)]),
                   (col(W), col(Vbc), [-1.0]),
                   (col(W2), col(VHl), [1.0])]
    mpairs = [(nodes(Psi), nodes(Psi), -occ * th),
              (nodes(PC), nodes(Psi_t), -np.ones(k)),
              (nodes(Y), nodes(Psi_l), lam_l + prob.mu),
              (nodes(Y), nodes(res.Psi_hat), -prob.mu * np.ones(k))]
    return shape_derivative(prob, kpairs, mpairs, F, rho - gam)


def forces_with_mesh_motion(F_fixed_mesh, gX, Wm):
    """F_a = F_a(fixed mesh) - sum_v Wm[v, a] dE/dX_v for a mesh whose node v
    moves by Wm[v, a] dR_a when nucleus a moves by dR_a."""
    return np.asarray(F_fixed_mesh) - np.einsum("va,vd->ad", Wm, gX)


def p2_midpoint_field(elems, D):
    """A nodal displacement field with every P2 edge node at the mean of its
    edge's vertex values (the vertices' values are kept)."""
    D = np.array(D, dtype=np.float64, copy=True)
    if elems.shape[1] == 10:
        for e, (a, b) in enumerate(fe.P2_EDGES):
            D[elems[:, 4 + e]] = 0.5 * (D[elems[:, a]] + D[elems[:, b]])
    return D
