"""Pins for one augmented-subspace step (Algorithm 3) of the oracle.

Brute force on tiny meshes (dense generalised eigensolves, numpy.linalg /
scipy.linalg used only as independent checking tools), Courant-Fischer
bounds, the fixed-point property, span invariance, orthonormality, charge
conservation, Anderson's least-squares property and agreement of a converged
run of Algorithm 3 with a direct dense SCF on the fine space."""
import numpy as np
import pytest
import scipy.linalg as sla

from ks_inputs import make_workload
from oracle.step import (KSProblem, ks_scf_step, initial_guess, anderson_mix, small_eig)
from oracle.xc import lda_xc


def _tiny_linear(n=6, k=1, n_H=4, mu=8.0):
    w = make_workload("hydrogen", n=n, k=k)
    w.n_H = n_H
    return KSProblem.from_workload(w, mu=mu)


def _tiny_nonlinear(n=6, order=1, n_H=3, mu=5.0, k=None):
    w = make_workload("small_molecule", n=n, order=order, k=k)
    w.n_H = n_H
    return KSProblem.from_workload(w, mu=mu)


def test_linear_step_obeys_courant_fischer_bounds():
    p = _tiny_linear(k=4)
    A = p.A_linear().toarray()
    lam_h = sla.eigh(A, p.M_II.toarray(), eigvals_only=True)[:4]
    th0, Psi = initial_guess(p, 4)
    r = ks_scf_step(p, Psi, th0, tol_solve=1e-13)
    assert r.inner_iters == 1
    assert np.all(lam_h <= r.lam + 1e-12)
    assert np.all(r.lam <= th0 + 1e-12)
    # repeated steps approach the discrete eigenvalues monotonically
    lam_prev = r.lam
    for _ in range(5):
        r = ks_scf_step(p, r.Psi, r.lam, tol_solve=1e-13)
        assert np.all(r.lam <= lam_prev + 1e-12) and np.all(lam_h <= r.lam + 1e-12)
        lam_prev = r.lam


def test_fixed_point_at_exact_discrete_eigenpairs():
    """Started at exact eigenpairs of (A, M), S psi = (lambda + mu) M psi, so
    psi_hat = psi and the Ritz step returns the same pairs."""
    p = _tiny_linear(k=2)
    A = p.A_linear().toarray()
    lam, V = sla.eigh(A, p.M_II.toarray())
    r = ks_scf_step(p, V[:, :2], lam[:2], tol_solve=1e-14)
    assert np.abs(r.lam - lam[:2]).max() < 1e-10
    assert np.abs(r.Psi_hat - V[:, :2]).max() < 1e-10
    d = r.rho_q - p.density(V[:, :2])
    assert np.sqrt(p.inner(d, d)) < 1e-9


def test_orthonormality_and_charge():
    p = _tiny_nonlinear(order=2, n=4)
    th0, Psi = initial_guess(p, 5)
    r = ks_scf_step(p, Psi, th0, tol_solve=1e-12, tol_inner=1e-11)
    G = r.Psi.T @ (p.M_II @ r.Psi)
    assert np.abs(G - np.eye(5)).max() < 1e-11
    assert abs(np.sum(p.dV * r.rho_q) - p.occ.sum()) < 1e-10
    # the output is an eigenpair of the projected pencil
    res = r.FA @ r.U - r.FB @ r.U * r.lam[None, :]
    assert np.abs(res).max() < 1e-9 * np.abs(r.FA).max()


def test_span_invariance_under_rhs_scaling():
    """Changing lambda^l rescales each BVP solution; the augmented space and
    therefore the step's output do not change."""
    p = _tiny_nonlinear(order=1, n=6)
    th0, Psi = initial_guess(p, 5)
    r1 = ks_scf_step(p, Psi, th0, tol_solve=1e-14, tol_inner=1e-12)
    r2 = ks_scf_step(p, Psi, th0 + np.array([0.1, 0.3, -0.2, 0.05, 0.7]), tol_solve=1e-14,
                     tol_inner=1e-12)
    assert np.abs(r1.lam - r2.lam).max() < 1e-9
    d = r1.rho_q - r2.rho_q
    assert np.sqrt(p.inner(d, d)) < 1e-8


def test_small_eig_invariant_to_basis_change():
    rng = np.random.default_rng(0)
    m, k = 12, 3
    Zb = rng.normal(size=(40, m))
    Mf = np.diag(rng.uniform(1, 2, 40))
    Af = rng.normal(size=(40, 40)); Af = Af + Af.T
    FA, FB = Zb.T @ Af @ Zb, Zb.T @ Mf @ Zb
    th, U, rank, _ = small_eig(FA, FB, k)
    Rm = rng.normal(size=(m, m))
    th2, U2, _, _ = small_eig(Rm.T @ FA @ Rm, Rm.T @ FB @ Rm, k)
    assert rank == m
    assert np.allclose(th, th2, rtol=1e-10)
    ref = sla.eigh(FA, FB, eigvals_only=True)[:k]
    assert np.allclose(th, ref, rtol=1e-10)
    # a duplicated column is dropped, not amplified
    Zd = np.hstack([Zb, Zb[:, :1]])
    th3, _, rank3, _ = small_eig(Zd.T @ Af @ Zd, Zd.T @ Mf @ Zd, k)
    assert rank3 == m and np.allclose(th3, th, rtol=1e-9)


def test_anderson_coefficients_minimise_residual_norm():
    rng = np.random.default_rng(2)
    wts = rng.uniform(0.5, 1.5, 30)
    inner = lambda a, b: float(np.sum(wts * a * b))
    hin = [rng.normal(size=30) for _ in range(4)]
    hout = [rng.normal(size=30) for _ in range(4)]
    beta = 0.7
    new = anderson_mix(hin, hout, inner, beta=beta, depth=5)
    F = [o - i for i, o in zip(hin, hout)]
    D = np.stack([F[-1] - F[j] for j in range(3)], 1) * np.sqrt(wts)[:, None]
    alpha, *_ = np.linalg.lstsq(D, F[-1] * np.sqrt(wts), rcond=None)
    rin = hin[-1] + sum(alpha[j] * (hin[j] - hin[-1]) for j in range(3))
    rout = hout[-1] + sum(alpha[j] * (hout[j] - hout[-1]) for j in range(3))
    assert np.allclose(new, beta * rout + (1 - beta) * rin, atol=1e-9)
    # first step: plain linear mixing
    one = anderson_mix(hin[:1], hout[:1], inner, beta=beta)
    assert np.allclose(one, beta * hout[0] + (1 - beta) * hin[0])


def _direct_dense_scf(p, k, tol=1e-12, beta=0.5, max_it=400):
    """Self-consistent field on the whole fine space with dense eigensolves."""
    A0 = (0.5 * p.K_II + p.Mext_II).toarray()
    Md = p.M_II.toarray()
    lam, V = sla.eigh(A0, Md)
    rho = p.density(V[:, :k])
    for it in range(max_it):
        wB = p.boundary_data(rho)
        VH, _ = p.hartree_nodes(rho, wB, 1e-14)
        _, vxc = lda_xc(rho, p.xc_mode)
        A = A0 + p.potential_matrix(p.at_quad(VH) + vxc).toarray()
        lam, V = sla.eigh(A, Md)
        rho_out = p.density(V[:, :k])
        d = rho_out - rho
        if np.sqrt(p.inner(d, d)) < tol:
            return lam[:k], rho_out, it
        rho = rho + beta * d
    raise RuntimeError("direct SCF did not converge")


@pytest.mark.slow
def test_converged_augmented_iteration_equals_direct_scf():
    p = _tiny_nonlinear(order=1, n=6, n_H=4, mu=4.0, k=2)
    k = 2
    lam_d, rho_d, _ = _direct_dense_scf(p, k)
    th, Psi = initial_guess(p, k)
    rho_prev = p.density(Psi)
    for step in range(300):
        r = ks_scf_step(p, Psi, th, tol_solve=1e-13, tol_inner=1e-12, tol_poisson=1e-14)
        d = r.rho_q - rho_prev
        Psi, th, rho_prev = r.Psi, r.lam, r.rho_q
        if np.sqrt(p.inner(d, d)) < 1e-11:
            break
    assert np.abs(th - lam_d).max() < 1e-8
    d = r.rho_q - rho_d
    assert np.sqrt(p.inner(d, d)) < 1e-8
    # at outer convergence the two energy expressions coincide
    E = r.energies
    assert abs(E["total"] - E["KS"]) < 1e-8


def test_inner_iteration_cap_keeps_energy_density_pairing():
    """When the inner iteration stops at its limit, the reported energies and
    the final pencil belong to one input density: nothing is mixed after the
    last pass.  With a limit of one pass that density is rho^l itself, and the
    Hartree energy 1/2 <V_H, rho_in> must equal the frozen-boundary form
    1/2 <rho, V_0[rho]> + <rho, V_bc> - 1/2 <rho^l, V_bc> at rho = rho^l, which
    is computed from two separate Poisson problems (zero-Dirichlet and
    harmonic lift)."""
    from oracle.step import step_energy
    p = _tiny_nonlinear(order=1, n=6)
    th0, Psi = initial_guess(p, 5)
    r1 = ks_scf_step(p, Psi, th0, tol_solve=1e-13, tol_inner=1e-14, tol_poisson=1e-14,
                     max_inner=1)
    assert r1.inner_iters == 1 and r1.extra["res_inner"] > 1e-14
    rho_l = r1.extra["rho_l"]
    assert np.array_equal(r1.extra["rho_in"], rho_l)
    e = step_energy(p, Psi, rho_l, rho_l, r1.extra["w_B"], tol_poisson=1e-14)
    assert abs(r1.energies["H_in"] - e["H_step"]) < 1e-10 * abs(e["H_step"])
    eps, vxc = lda_xc(rho_l, p.xc_mode)
    assert abs(r1.energies["xc_in"] - p.inner(eps, rho_l)) < 1e-12 * abs(r1.energies["xc_in"])
    # a later cap: the final pencil was built from the returned rho_in
    r3 = ks_scf_step(p, Psi, th0, tol_solve=1e-13, tol_inner=1e-14, tol_poisson=1e-14,
                     max_inner=3)
    assert r3.inner_iters == 3
    rin = r3.extra["rho_in"]
    VH, _ = p.hartree_nodes(rin, r3.extra["w_B"], 1e-14)
    _, vxc = lda_xc(rin, p.xc_mode)
    Z = r3.extra["Z"]
    FA = r3.FA_L + Z.T @ (p.potential_matrix(p.at_quad(VH) + vxc) @ Z)
    assert np.abs(FA - r3.FA).max() < 1e-9 * np.abs(r3.FA).max()
    assert abs(r3.energies["H_in"] - 0.5 * p.inner(p.at_quad(VH), rin)) < 1e-10 * abs(r3.energies["H_in"])


def test_initial_guess_on_nested_mesh_is_the_coarse_mesh_problem():
    """With V_ext = 0 (a zero nuclear charge) and a fine mesh that refines
    the coarse Kuhn mesh T_H, span(I_H^h) is the coarse P1 space itself, so
    the Ritz pairs of initial_guess are the eigenpairs of (1/2 K_H, M_H)
    assembled on T_H (eq. st5: A_H = I^T A_h I) and every orbital is a
    coarse eigenvector interpolated to the fine nodes.  A wrong operator,
    basis or ordering in initial_guess fails this."""
    from ks_inputs.mesh import freudenthal_mesh
    from ks_inputs.quadrature import rule_for_order
    L, nH, k = 4.0, 3, 4
    coarse = freudenthal_mesh(nH, L, 1)
    pc = KSProblem(order=1, coords=coarse.coords, elems=coarse.elems, dirichlet=coarse.dirichlet,
                   quad=rule_for_order(1), Z=np.array([0.0]), R=np.full((1, 3), 0.1),
                   occ=np.ones(k), L=L, n_H=nH, mu=1.0, hartree=False, xc_mode="none")
    pc.setup()
    lam_H = sla.eigh(0.5 * pc.K_II.toarray(), pc.M_II.toarray(), eigvals_only=True)[:k]
    for order in (1, 2):
        fine = freudenthal_mesh(2 * nH, L, order)
        pf = KSProblem(order=order, coords=fine.coords, elems=fine.elems, dirichlet=fine.dirichlet,
                       quad=rule_for_order(order), Z=np.array([0.0]), R=np.full((1, 3), 0.1),
                       occ=np.ones(k), L=L, n_H=nH, mu=1.0, hartree=False, xc_mode="none")
        pf.setup()
        assert np.abs(pf.vext_q).max() == 0.0
        th, Psi = initial_guess(pf, k)
        assert np.abs(th - lam_H).max() < 1e-10 * np.abs(lam_H).max()
        # the orbitals are coarse functions solving the coarse problem
        U = np.linalg.lstsq(pf.P, Psi, rcond=None)[0]
        assert np.abs(pf.P @ U - Psi).max() < 1e-10
        Kc, Mc = 0.5 * pc.K_II.toarray(), pc.M_II.toarray()
        assert np.abs(Kc @ U - (Mc @ U) * th[None, :]).max() < 1e-10
        assert np.abs(Psi.T @ (pf.M_II @ Psi) - np.eye(k)).max() < 1e-10


def test_conditioned_pencil_equals_the_plain_formulation():
    """The oracle M-orthogonalises psi_hat against span(P), scales the pencil
    and drops the shift mu (its conditioning devices).  The plain form of the
    step -- Z = [P | psi_hat] with psi_hat from a dense solve, the shifted
    pencil (Z^T (A + mu M) Z, Z^T M Z), no scaling -- spans the same space and
    must give the same Ritz values: in the linear case directly, in the
    nonlinear case with the step's final Hamiltonian."""
    for p, kw in ((_tiny_linear(k=3), dict(tol_solve=1e-14)),
                  (_tiny_nonlinear(order=1, n=5), dict(tol_solve=1e-14, tol_inner=1e-12, tol_poisson=1e-14))):
        k = 3 if not p.hartree else 5
        th0, Psi = initial_guess(p, k)
        r = ks_scf_step(p, Psi, th0, **kw)
        Mm = p.M_II.toarray()
        S = r.extra["S"].toarray()
        Psi_hat = np.linalg.solve(S, (Mm @ Psi) * (th0 + p.mu)[None, :])
        A = p.A_linear()
        if p.hartree or p.xc_mode != "none":
            A = A + p.potential_matrix(r.extra["vnl_in"])
        A = A.toarray()
        Z = np.hstack([p.P, Psi_hat])
        lam = sla.eigh(Z.T @ (A + p.mu * Mm) @ Z, Z.T @ Mm @ Z, eigvals_only=True)[:k] - p.mu
        assert np.abs(lam - r.lam).max() < 1e-9 * np.abs(lam).max()
