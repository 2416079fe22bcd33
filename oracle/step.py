"""ORACLE (test infrastructure only): one iteration of the augmented subspace
method (Algorithm 3, Sec. 3.3) with its inner nonlinear iteration.

One step, given (Lambda^l, Psi^l):
  1. rho^l = sum_i f_i psi_i^2 at the quadrature points; V_H(rho^l) with the
     multipole data w_D(rho^l); V_xc(rho^l);
     S = 1/2 K + M[V_ext + V_H + V_xc] + mu M            (Sec. 3.3, H-tilde)
  2. the N boundary value problems S psi_hat_i = (lambda_i + mu) M psi_i
                                               (eq. Aux_Linear_Problem)
  3. Z = [P | Psi_hat]: coarse basis interpolated to the fine mesh plus the
     BVP solutions (M-orthogonalised against span P); F_B = Z^T M Z and
     F_A^L = Z^T (1/2 K + M[V_ext]) Z assembled once (eqs. st1-st7,
     consistent-Galerkin reading below)
  4. the small Kohn-Sham problem in span(Z) (eq. Nonlinear_Eig_Hh), solved by
     a nonlinear iteration with Anderson mixing on the density (Sec. 4):
     F_A = F_A^L + Z^T M[V_H(rho_in) + V_xc(rho_in)] Z, lowest k pairs of the
     pencil (F_A, F_B), Psi = Z U, rho_out, mix, until ||rho_out - rho_in||_0
     < tol_inner
  5. Psi^{l+1} = Z U, energies.

Readings (the paper leaves these open):
  * F_A = Z^T A Z and F_B = Z^T M Z on the fine mesh with Z = [I_H^h | Psi_hat]
    (A_H = I^T A I per eq. st5 and its mass analogue), so the augmented space
    is a subspace of the fine space.
  * w_D is computed from the step's input density rho^l and held fixed through
    the inner iteration.
  * density update with occupations: rho = sum f_i psi_i^2.
  * the projected pencil leaves out the shift mu of eq. st3 (F_A - mu F_B has
    the same eigenvectors and eigenvalues lambda = theta - mu; forming it
    directly avoids cancelling mu ~ 1e3..1e5 against lambda ~ 1).
  * small eigenproblem: diagonal scaling, canonical orthogonalisation of F_B
    (drop eigenvalues below 1e-12 of the largest), then a symmetric
    eigensolve; the largest-magnitude entry of every column of U is made
    positive.
  * Anderson inner product: the quadrature L2 inner product <a, b> =
    sum_eq dV_eq a_eq b_eq; first mixing step is linear with beta; Tikhonov
    term 1e-12 trace(G) on the normal equations.
  * energies: E_total = sum f_i lambda_i - <V_H/2 + V_xc, rho_in> +
    <rho_in, eps_xc(rho_in)> + E_nn (Sec. 3.1 with occupations, evaluated on
    the density that built the final Hamiltonian) and the functional
    E_KS(Psi^{l+1}) of Sec. 2 with the step's frozen-boundary Hartree term.
"""
from dataclasses import dataclass, field
import numpy as np
import scipy.sparse as sp

from . import fe
from .xc import lda_xc
from .hartree import density_moments, multipole_boundary
from .solvers import jacobi_pcg
from .coarse import coarse_interpolation, interpolation_in_mesh


@dataclass
class KSProblem:
    """Per-mesh data of the discrete problem (fixed for a mesh)."""
    order: int
    coords: np.ndarray
    elems: np.ndarray
    dirichlet: np.ndarray
    quad: object
    Z: np.ndarray
    R: np.ndarray
    occ: np.ndarray
    L: float
    n_H: int
    mu: float
    hartree: bool = True
    xc_mode: str = "x_pz81"
    quad_factor: float = 0.5
    coarse: object = None        # a nonnested coarse P1 mesh (None: uniform n_H)
    # derived
    n_nodes: int = 0
    interior: np.ndarray = None
    boundary: np.ndarray = None
    J: np.ndarray = None
    det: np.ndarray = None
    gl: np.ndarray = None
    dV: np.ndarray = None
    x_q: np.ndarray = None
    vext_q: np.ndarray = None
    K: object = None
    M: object = None
    K_II: object = None
    K_IB: object = None
    M_II: object = None
    Mext_II: object = None
    P: np.ndarray = None
    extra: dict = field(default_factory=dict)

    @classmethod
    def from_workload(cls, w, mu=None, quad_factor=0.5, coarse=None):
        p = cls(order=w.mesh.order, coords=w.mesh.coords, elems=w.mesh.elems,
                dirichlet=w.mesh.dirichlet, quad=w.quad, Z=w.atoms.Z, R=w.atoms.R,
                occ=w.occ, L=w.mesh.L, n_H=w.n_H,
                mu=w.mu_paper if mu is None else mu, hartree=w.hartree,
                xc_mode="x_pz81" if w.xc else "none", quad_factor=quad_factor, coarse=coarse)
        p.setup()
        return p

    def setup(self):
        self.n_nodes = self.coords.shape[0]
        self.interior = np.flatnonzero(self.dirichlet == 0)
        self.boundary = np.flatnonzero(self.dirichlet != 0)
        self.J, self.det, self.gl = fe.element_geometry(self.coords, self.elems)
        self.dV = fe.quad_weights(self.det, self.quad.w)
        self.x_q = fe.quad_points(self.coords, self.elems, self.quad.bary)
        self.vext_q = external_potential(self.x_q, self.Z, self.R)
        Ke = fe.element_matrices(self.order, self.quad, self.det, self.gl, kind="stiffness")
        Me = fe.element_matrices(self.order, self.quad, self.det, self.gl, kind="mass")
        MVe = fe.element_matrices(self.order, self.quad, self.det, self.gl, V=self.vext_q,
                                  kind="potential")
        self.K = fe.assemble(self.n_nodes, self.elems, Ke)
        self.M = fe.assemble(self.n_nodes, self.elems, Me)
        Mext = fe.assemble(self.n_nodes, self.elems, MVe)
        I, B = self.interior, self.boundary
        self.K_II = fe.restrict(self.K, I, I)
        self.K_IB = fe.restrict(self.K, I, B)
        self.M_II = fe.restrict(self.M, I, I)
        self.Mext_II = fe.restrict(Mext, I, I)
        if self.coarse is None:
            self.P = coarse_interpolation(self.coords[I], self.L, self.n_H)
        else:  # Sec. 3.2: coarse space on a nonnested mesh
            self.P = interpolation_in_mesh(self.coords[I], self.coarse.coords, self.coarse.elems,
                                           self.coarse.dirichlet)

    def moved(self, coords):
        """Copy of the problem with the mesh nodes at `coords` (same
        connectivity) and the same coarse interpolation matrix P: the coarse
        space is carried along by the moving mesh."""
        import copy
        q = copy.copy(self)
        q.coords = np.asarray(coords, dtype=np.float64)
        P = self.P
        q.setup()
        q.P = P
        return q

    def with_external(self, vext_q=None, R=None):
        """Copy of the problem with another external potential at the
        quadrature points (or nuclei moved to R, which also changes E_nn);
        the mesh and everything else are shared."""
        import copy
        q = copy.copy(self)
        if R is not None:
            q.R = np.asarray(R, dtype=np.float64).reshape(-1, 3)
            vext_q = external_potential(self.x_q, q.Z, q.R)
        q.vext_q = np.asarray(vext_q, dtype=np.float64)
        MVe = fe.element_matrices(self.order, self.quad, self.det, self.gl, V=q.vext_q,
                                  kind="potential")
        q.Mext_II = fe.restrict(fe.assemble(self.n_nodes, self.elems, MVe), self.interior,
                                self.interior)
        return q

    # --- operators --------------------------------------------------------
    @property
    def N(self):
        return self.interior.shape[0]

    def A_linear(self):
        """A^L = 1/2 K + M[V_ext] (eq. st3 without the shift)."""
        return (0.5 * self.K_II + self.Mext_II).tocsr()

    def potential_matrix(self, V_q):
        """M[V]_II for quadrature values V_q (eq. st4)."""
        MVe = fe.element_matrices(self.order, self.quad, self.det, self.gl, V=V_q,
                                  kind="potential")
        return fe.restrict(fe.assemble(self.n_nodes, self.elems, MVe), self.interior,
                           self.interior)

    def to_nodes(self, X):
        """Interior values [N](k) -> all nodes, zero on the Dirichlet boundary."""
        out = np.zeros((self.n_nodes,) + X.shape[1:])
        out[self.interior] = X
        return out

    def density(self, Psi):
        return fe.density_at_quad(self.order, self.quad, self.elems, self.to_nodes(Psi),
                                  self.occ)

    def inner(self, a, b):
        """<a, b> = sum_eq dV_eq a_eq b_eq (quadrature L2 inner product)."""
        return float(np.sum(self.dV * a * b))

    def E_nn(self):
        """E_nn = sum_{k<j} Z_j Z_k / |R_j - R_k| (Sec. 3.1)."""
        e = 0.0
        for j in range(len(self.Z)):
            for k in range(j):
                e += self.Z[j] * self.Z[k] / np.linalg.norm(self.R[j] - self.R[k])
        return e

    # --- Hartree ------------------------------------------------------------
    def boundary_data(self, rho_q):
        """w_D(rho) at the boundary nodes (eq. bd)."""
        if not self.hartree:
            return np.zeros(self.boundary.shape[0])
        Q, c, p, q = density_moments(rho_q, self.x_q, self.dV)
        return multipole_boundary(self.coords[self.boundary], Q, c, p, q, self.quad_factor)

    def hartree_nodes(self, rho_q, w_B, tol=1e-12):
        """Nodal V_H for density rho_q with boundary values w_B."""
        if not self.hartree:
            return np.zeros(self.n_nodes), 0
        load = fe.load_vector(self.order, self.quad, self.elems, self.det, self.n_nodes,
                              rho_q)[self.interior]
        rhs = 4.0 * np.pi * load - self.K_IB @ w_B
        VI, it, _ = jacobi_pcg(self.K_II, rhs, None, tol=tol, max_iter=200000)
        V = np.zeros(self.n_nodes)
        V[self.interior] = VI
        V[self.boundary] = w_B
        return V, int(it[0])

    def at_quad(self, U_nodes):
        return fe.eval_at_quad(self.order, self.quad, self.elems, U_nodes)


def external_potential(x_q, Z, R):
    """V_ext(x) = - sum_k Z_k / |x - R_k| (Sec. 2)."""
    v = np.zeros(x_q.shape[:-1])
    for z, r in zip(Z, R):
        v -= z / np.linalg.norm(x_q - r, axis=-1)
    return v


def small_eig(FA, FB, k, drop=1e-12):
    """Lowest k eigenpairs of F_A u = lambda F_B u (eq. st1).  The pencil is
    first scaled by D = diag(F_B)^{-1/2} (the columns of Z differ in size by
    orders of magnitude), then F_B is canonically orthogonalised (eigenvalues
    below ``drop`` times the largest are discarded) and the reduced symmetric
    problem is solved.  Returns (lambda[k], U[m][k], rank, lambda_all)."""
    d = 1.0 / np.sqrt(np.diag(FB))
    FBs = d[:, None] * FB * d[None, :]
    FAs = d[:, None] * FA * d[None, :]
    s, V = np.linalg.eigh(0.5 * (FBs + FBs.T))
    keep = s > drop * s.max()
    X = V[:, keep] / np.sqrt(s[keep])[None, :]
    C = X.T @ (0.5 * (FAs + FAs.T)) @ X
    th, W = np.linalg.eigh(0.5 * (C + C.T))
    U = d[:, None] * (X @ W[:, :k])
    for j in range(U.shape[1]):
        i = np.argmax(np.abs(U[:, j]))
        if U[i, j] < 0:
            U[:, j] = -U[:, j]
    return th[:k], U, int(keep.sum()), th


def anderson_mix(hist_in, hist_out, inner, beta=0.7, depth=5):
    """Next input density from the history (oldest first) of input/output
    densities, Sec. 4 (eqs. mix2-mix6): alpha minimises ||F~|| over the
    last ``depth`` iterates; rho_in^{m+1} = beta rho~_out + (1-beta) rho~_in."""
    hi = hist_in[-depth:]
    ho = hist_out[-depth:]
    Fm = ho[-1] - hi[-1]
    nh = len(hi) - 1
    if nh == 0:
        return beta * ho[-1] + (1.0 - beta) * hi[-1]
    D = [Fm - (ho[j] - hi[j]) for j in range(nh)]
    G = np.array([[inner(D[j], D[l]) for l in range(nh)] for j in range(nh)])
    c = np.array([inner(D[j], Fm) for j in range(nh)])
    G = G + 1e-12 * max(np.trace(G), 1e-300) * np.eye(nh)
    alpha = np.linalg.solve(G, c)
    rin = hi[-1] + sum(alpha[j] * (hi[j] - hi[-1]) for j in range(nh))
    rout = ho[-1] + sum(alpha[j] * (ho[j] - ho[-1]) for j in range(nh))
    return beta * rout + (1.0 - beta) * rin


def initial_guess(prob, k):
    """Ritz pairs of (1/2 K + M[V_ext], M) in the interpolated coarse space
    span(P): a stand-in for the coarse-mesh SCF stage of Algorithm 2."""
    P = prob.P
    FA = P.T @ (prob.A_linear() @ P)
    FB = P.T @ (prob.M_II @ P)
    th, U, _, _ = small_eig(FA, FB, k)
    return th, P @ U


def block_solve(prob, S, Psi, lam, tol=1e-8, max_iter=10000):
    """The N linear problems of Algorithm 3 (eq. Aux_Linear_Problem):
    S psi_hat_i = (lambda_i + mu) M psi_i, started at psi_i."""
    B = (prob.M_II @ Psi) * (lam + prob.mu)[None, :]
    return jacobi_pcg(S, B, Psi, tol=tol, max_iter=max_iter)


@dataclass
class StepResult:
    Psi: np.ndarray
    lam: np.ndarray
    rho_q: np.ndarray
    Psi_hat: np.ndarray
    theta_all: np.ndarray
    U: np.ndarray
    FA: np.ndarray
    FB: np.ndarray
    FA_L: np.ndarray
    energies: dict
    inner_iters: int
    solve_iters: np.ndarray
    solve_relres: np.ndarray
    rank: int
    extra: dict


def ks_scf_step(prob, Psi, lam, tol_solve=1e-8, tol_inner=1e-8, tol_poisson=1e-12,
                max_inner=50, anderson_depth=5, anderson_beta=0.7, want_eks=True, w_B=None):
    """One step; w_B (optional) replaces the multipole boundary data of the
    input density, for steps whose boundary data are held fixed."""
    Psi = np.asarray(Psi, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    k = Psi.shape[1]
    occ = prob.occ
    nonlinear = prob.hartree or prob.xc_mode != "none"
    # 1. Hamiltonian of the step's input density
    rho_l = prob.density(Psi)
    w_B = prob.boundary_data(rho_l) if w_B is None else np.asarray(w_B, dtype=np.float64)
    VH_l, _ = prob.hartree_nodes(rho_l, w_B, tol_poisson)
    eps_l, vxc_l = lda_xc(rho_l, prob.xc_mode)
    veff = prob.vext_q + prob.at_quad(VH_l) + vxc_l
    S = (0.5 * prob.K_II + prob.potential_matrix(veff) + prob.mu * prob.M_II).tocsr()
    # 2. boundary value problems
    Psi_hat, its, rr = block_solve(prob, S, Psi, lam, tol=tol_solve)
    # 3. augmented subspace and the fixed blocks.  Psi_hat is M-orthogonalised
    #    against span(P) first (same span, so the same Ritz pairs): with the
    #    large shift mu, Psi_hat differs from a coarse-space function only by
    #    O(1/mu), and forming that difference on the fine vectors keeps the
    #    pencil well conditioned.
    G_PP = prob.P.T @ (prob.M_II @ prob.P)
    T = np.linalg.solve(G_PP, prob.P.T @ (prob.M_II @ Psi_hat))
    Psi_t = Psi_hat - prob.P @ T
    Z = np.hstack([prob.P, Psi_t])
    AL = prob.A_linear()
    FB = Z.T @ (prob.M_II @ Z)
    FA_L = Z.T @ (AL @ Z)
    # 4. inner nonlinear iteration
    rho_in = rho_l.copy()
    hist_in, hist_out = [], []
    inner_iters = 0
    for it in range(max_inner):
        inner_iters = it + 1
        if nonlinear:
            VH, _ = prob.hartree_nodes(rho_in, w_B, tol_poisson)
            eps_in, vxc_in = lda_xc(rho_in, prob.xc_mode)
            VH_q = prob.at_quad(VH)
            MNL = prob.potential_matrix(VH_q + vxc_in)
            FA = FA_L + Z.T @ (MNL @ Z)
        else:
            VH_q = np.zeros_like(rho_in)
            eps_in, vxc_in = lda_xc(rho_in, "none")
            FA = FA_L
        th, U, rank, th_all = small_eig(FA, FB, k)
        Psi_new = Z @ U
        rho_out = prob.density(Psi_new)
        res = np.sqrt(max(prob.inner(rho_out - rho_in, rho_out - rho_in), 0.0))
        # the last permitted pass mixes nothing: the energies below pair
        # rho_in with the potentials it produced (Sec. 3.1)
        if not nonlinear or res < tol_inner or it == max_inner - 1:
            break
        hist_in.append(rho_in)
        hist_out.append(rho_out)
        rho_in = anderson_mix(hist_in, hist_out, prob.inner, anderson_beta, anderson_depth)
    lam_new = th
    # 5. energies
    E = {}
    E["band"] = float(np.sum(occ * lam_new))
    E["H_in"] = 0.5 * prob.inner(VH_q, rho_in)
    E["xc_in"] = prob.inner(eps_in, rho_in)
    E["vxc_rho_in"] = prob.inner(vxc_in, rho_in)
    E["nn"] = prob.E_nn()
    E["total"] = E["band"] - E["H_in"] - E["vxc_rho_in"] + E["xc_in"] + E["nn"]
    if want_eks:
        E.update(step_energy(prob, Psi_new, rho_out, rho_l, w_B, tol_poisson))
    return StepResult(Psi=Psi_new, lam=lam_new, rho_q=rho_out, Psi_hat=Psi_hat,
                      theta_all=th_all, U=U, FA=FA, FB=FB, FA_L=FA_L, energies=E,
                      inner_iters=inner_iters, solve_iters=its, solve_relres=rr, rank=rank,
                      extra={"S": S, "w_B": w_B, "rho_l": rho_l, "rho_in": rho_in,
                             "Z": Z, "res_inner": res, "vnl_in": VH_q + vxc_in,
                             "G_PP": G_PP})


def step_energy(prob, Psi, rho, rho_l, w_B, tol_poisson=1e-12):
    """Functional form (Sec. 2) of the energy of Psi with the step's frozen
    Hartree boundary data: with V_0 the zero-Dirichlet Poisson solution and
    V_bc the discrete harmonic lift of w_B,
      E_H^step = 1/2 <rho, V_0[rho]> + <rho, V_bc> - 1/2 <rho^l, V_bc>,
    which equals 1/2 <rho, V_H> at rho = rho^l and whose rho-derivative is
    V_H = V_0[rho] + V_bc."""
    out = {}
    kin = 0.5 * float(np.sum(prob.occ * np.sum(Psi * (prob.K_II @ Psi), axis=0)))
    out["kin"] = kin
    out["ext"] = prob.inner(prob.vext_q, rho)
    if prob.hartree:
        V0, _ = prob.hartree_nodes(rho, np.zeros_like(w_B), tol_poisson)
        Vbc, _ = prob.hartree_nodes(np.zeros_like(rho), w_B, tol_poisson)
        V0q, Vbcq = prob.at_quad(V0), prob.at_quad(Vbc)
        eh = 0.5 * prob.inner(rho, V0q) + prob.inner(rho, Vbcq) - 0.5 * prob.inner(rho_l, Vbcq)
    else:
        eh = 0.0
    out["H_step"] = eh
    eps, _ = lda_xc(rho, prob.xc_mode)
    out["xc"] = prob.inner(rho, eps)
    out["KS"] = kin + out["ext"] + eh + out["xc"] + prob.E_nn()
    return out


def step_backward(prob, res, tol=1e-13):
    """Gradient of E_KS(Psi^{l+1}) of one step with respect to V_ext at the
    quadrature points and the nuclear forces, the step's inputs (Psi^l,
    lambda^l, rho^l and the boundary data) held fixed.

    With the inner iteration converged, Psi^{l+1} is a stationary point of
    E_KS over span(Z) with Psi^T M Psi = I, so (envelope theorem) only the
    explicit V_ext term and the dependence of Z on V_ext through the BVPs
    remain:
      R = A Psi - M Psi Theta           (A: Hamiltonian of the final inner step)
      dE/dZ = 2 R F U^T                 (F = diag(occupations))
      Psi_bar_tilde = its Psi-tilde columns; Psi_bar_hat = Psi_bar_tilde
          - M P G^{-1} P^T Psi_bar_tilde   (chain rule of the M-orthogonalisation)
      S Y = Psi_bar_hat                 (adjoint BVPs; S symmetric)
      dPsi_hat = -S^{-1} M[dV] Psi_hat  =>  dE = -sum_i Y_i^T M[dV] psi_hat_i
    so  g_q = w_q |J| (rho_q - sum_i Y_i(x_q) psi_hat_i(x_q)),
    and F_k = -sum_q g_q dV_ext(x_q)/dR_k - dE_nn/dR_k with
    dV_ext/dR_k = -Z_k (x - R_k)/|x - R_k|^3."""
    k = res.Psi.shape[1]
    NH = prob.P.shape[1]
    Psi, U, th = res.Psi, res.U, res.lam
    A = (prob.A_linear() + prob.potential_matrix(res.extra["vnl_in"])).tocsr() \
        if (prob.hartree or prob.xc_mode != "none") else prob.A_linear()
    R = A @ Psi - (prob.M_II @ Psi) * th[None, :]
    bar_t = 2.0 * (R * prob.occ[None, :]) @ U[NH:NH + k, :].T
    G = res.extra["G_PP"]
    bar_h = bar_t - prob.M_II @ (prob.P @ np.linalg.solve(G, prob.P.T @ bar_t))
    Y, its, rr = jacobi_pcg(res.extra["S"], bar_h, None, tol=tol, max_iter=100000)
    Yq = prob.at_quad(prob.to_nodes(Y))
    Hq = prob.at_quad(prob.to_nodes(res.Psi_hat))
    g = prob.dV * (res.rho_q - np.einsum("eqk,eqk->eq", Yq, Hq))
    # forces
    F = np.zeros((len(prob.Z), 3))
    for a, (z, r) in enumerate(zip(prob.Z, prob.R)):
        d = prob.x_q - r[None, None, :]
        dist3 = np.sum(d * d, axis=-1) ** 1.5
        dV = -z * d / dist3[..., None]          # dV_ext/dR_a at every point
        F[a] = -np.einsum("eq,eqd->d", g, dV)
        for b, (zb, rb) in enumerate(zip(prob.Z, prob.R)):
            if b != a:
                dr = r - rb
                F[a] += z * zb * dr / np.linalg.norm(dr) ** 3   # -dE_nn/dR_a
    return g, F, {"adjoint_iters": its, "R_norm": np.linalg.norm(R)}
