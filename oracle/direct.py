"""ORACLE (test infrastructure only): the "direct" method that the paper's
experiments compare Algorithm 3 with (Sec. 4: the self-consistent field
iteration solved directly on the fine finite element space).

Every iteration takes the input density rho_in, builds the linear Kohn-Sham
operator of Sec. 3.1 on the fine space,
    H(rho_in) = 1/2 K + M[V_ext + V_H(rho_in) + V_xc(rho_in)],
with V_H solved from the Poisson problem whose multipole boundary data w_D is
computed from rho_in itself (eq. bd), takes the lowest k eigenpairs of
(H, M), forms rho_out = sum_i f_i psi_i^2, and stops when
||rho_out - rho_in||_0 < tol; otherwise the next input density comes from
Anderson mixing (Sec. 4, eqs. mix2-mix6; depth 5, beta 0.7 in the paper).
The energy is the one of Sec. 3.1 evaluated on the density that built the
final operator, as for one step of Algorithm 3.

The eigenpairs come from scipy: a dense generalised eigensolve for small
problems, else a sparse shift-and-invert Lanczos (ARPACK) about a shift
below the lowest eigenvalue.  A fixed point of this iteration is a fixed
point of Algorithm 3 (same discrete Kohn-Sham equations).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from .xc import lda_xc
from .step import anderson_mix


def lowest_eigenpairs(H, M, k, dense_limit=2500, shift=None):
    """Lowest k eigenpairs of the symmetric pencil (H, M), M positive definite."""
    n = H.shape[0]
    if n <= dense_limit:
        lam, V = sla.eigh(H.toarray(), M.toarray(), subset_by_index=[0, k - 1])
        return lam, V
    if shift is None:
        shift = float(H.diagonal().min() / M.diagonal().max()) - 1.0
    lam, V = spla.eigsh(H.tocsc(), k=k, M=M.tocsc(), sigma=shift, which="LM", tol=1e-13)
    order = np.argsort(lam)
    return lam[order], V[:, order]


def direct_scf(prob, k, Psi0=None, tol=1e-8, max_it=300, depth=5, beta=0.7, tol_poisson=1e-12,
               dense_limit=2500):
    """Direct SCF on the fine space.  Psi0 [N][k] (None: the lowest k
    eigenvectors of 1/2 K + M[V_ext]).  Returns a dict with lam, Psi, rho
    (the output density), rho_in, energies, iters and res."""
    AL = prob.A_linear()
    M = prob.M_II
    if Psi0 is None:
        _, Psi0 = lowest_eigenpairs(AL, M, k, dense_limit)
    rho_in = prob.density(np.asarray(Psi0, dtype=np.float64))
    hist_in, hist_out = [], []
    shift = None
    res, it = np.inf, 0
    for it in range(1, max_it + 1):
        w_B = prob.boundary_data(rho_in)
        VH, _ = prob.hartree_nodes(rho_in, w_B, tol_poisson)
        VH_q = prob.at_quad(VH)
        eps_in, vxc_in = lda_xc(rho_in, prob.xc_mode)
        H = (AL + prob.potential_matrix(VH_q + vxc_in)).tocsr()
        lam, Psi = lowest_eigenpairs(H, M, k, dense_limit, shift)
        shift = float(lam[0]) - 1.0
        rho_out = prob.density(Psi)
        d = rho_out - rho_in
        res = np.sqrt(max(prob.inner(d, d), 0.0))
        if res < tol or it == max_it:
            break
        hist_in.append(rho_in)
        hist_out.append(rho_out)
        rho_in = anderson_mix(hist_in, hist_out, prob.inner, beta, depth)
    occ = prob.occ
    E = {"band": float(np.sum(occ * lam)), "H_in": 0.5 * prob.inner(VH_q, rho_in),
         "xc_in": prob.inner(eps_in, rho_in), "vxc_rho_in": prob.inner(vxc_in, rho_in),
         "nn": prob.E_nn()}
    E["total"] = E["band"] - E["H_in"] - E["vxc_rho_in"] + E["xc_in"] + E["nn"]
    return {"lam": lam, "Psi": Psi, "rho": rho_out, "rho_in": rho_in, "energies": E,
            "iters": it, "res": res}
