"""Pins for the oracle's LDA, Hartree/multipole, coarse interpolation and
hydrogen-like eigenvalues against closed forms and textbook identities."""
import numpy as np
import pytest
from scipy.special import erf
import scipy.sparse.linalg as sla

from ks_inputs import make_workload, freudenthal_mesh
from ks_inputs.quadrature import rule_for_order
from oracle import fe
from oracle.xc import lda_xc
from oracle.hartree import density_moments, multipole_boundary
from oracle.coarse import coarse_interpolation
from oracle.solvers import jacobi_pcg
from oracle.step import KSProblem, external_potential


# --------------------------------------------------------------------- LDA
def test_exchange_potential_is_derivative_of_energy_density():
    rho = np.logspace(-6, 2, 50)
    e, v = lda_xc(rho, "x_only")
    assert np.allclose(v, 4.0 / 3.0 * e, rtol=1e-14)
    # V_x = -(3 rho / pi)^{1/3} is exactly -1 at rho = pi/3
    _, v1 = lda_xc(np.array([np.pi / 3.0]), "x_only")
    assert abs(v1[0] + 1.0) < 1e-15


@pytest.mark.parametrize("rs", [0.05, 0.2, 0.5, 0.9, 1.1, 2.0, 5.0, 20.0])
def test_correlation_potential_is_derivative_of_energy_density(rs):
    """V_c = d(rho eps_c)/d rho, by central differences in rho (away from the
    r_s = 1 branch switch)."""
    rho = 3.0 / (4.0 * np.pi * rs ** 3)
    h = 1e-5 * rho
    ex_p, _ = lda_xc(np.array([rho + h]), "x_only")
    ex_m, _ = lda_xc(np.array([rho - h]), "x_only")
    e_p, _ = lda_xc(np.array([rho + h]))
    e_m, _ = lda_xc(np.array([rho - h]))
    ec_p = e_p - ex_p
    ec_m = e_m - ex_m
    fd = ((rho + h) * ec_p - (rho - h) * ec_m) / (2 * h)
    e0, v0 = lda_xc(np.array([rho]))
    ex0, vx0 = lda_xc(np.array([rho]), "x_only")
    assert abs((v0 - vx0)[0] - fd[0]) < 1e-8 * max(1.0, abs(fd[0]))


def test_correlation_branch_gap_at_rs_one_is_as_printed():
    """The printed constants leave a small jump at r_s = 1 (eps_c ~3e-5);
    the high-density branch applies for r_s < 1, the other at r_s = 1."""
    def ec(rs):
        rho = 3.0 / (4.0 * np.pi * rs ** 3)
        e, _ = lda_xc(np.array([rho]))
        ex, _ = lda_xc(np.array([rho]), "x_only")
        return (e - ex)[0]
    lo = 0.0311 * np.log(1.0 - 1e-12) - 0.048
    assert abs(ec(1.0 - 1e-9) - (-0.048 - 0.0116)) < 1e-8
    assert abs(ec(1.0) - (-0.1423 / (1 + 1.0529 + 0.3334))) < 1e-15
    assert 1e-5 < abs(ec(1.0) - ec(1.0 - 1e-9)) < 1e-4
    assert np.isfinite(lo)


def _golden_pz81():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "lda_pz81_constants.txt")
    vals = {}
    for line in open(path):
        line = line.split("#")[0].split()
        if len(line) == 2:
            vals[line[0]] = float(line[1])
    return vals


def test_correlation_uses_the_printed_constants():
    """The oracle's correlation energy at r_s = 0.5 (first branch) and r_s = 4
    (second branch) equals the paper's formulas with the constants read from
    the golden file (Sec. 3.1), and the low-density branch's energy and
    potential approach zero like gamma / (beta_2 r_s) as r_s grows."""
    g = _golden_pz81()
    assert len(g) == 7

    def ec_vc(rs):
        rho = 3.0 / (4.0 * np.pi * rs ** 3)
        e, v = lda_xc(np.array([rho]))
        ex, vx = lda_xc(np.array([rho]), "x_only")
        return (e - ex)[0], (v - vx)[0]

    rs = 0.5
    ec, _ = ec_vc(rs)
    assert abs(ec - (g["A"] * np.log(rs) + g["B"] + g["C"] * rs * np.log(rs) + g["D"] * rs)) < 1e-15
    rs = 4.0
    ec, vc = ec_vc(rs)
    den = 1 + g["beta_1"] * np.sqrt(rs) + g["beta_2"] * rs
    assert abs(ec - g["gamma"] / den) < 1e-15
    rs = 1e8
    ec, vc = ec_vc(rs)
    assert abs(ec * g["beta_2"] * rs / g["gamma"] - 1) < 1e-3
    assert abs(vc * g["beta_2"] * rs / g["gamma"] - 4.0 / 3.0) < 1e-3


def test_xc_vanishes_at_zero_density():
    e, v = lda_xc(np.array([0.0, 1e-31, -1e-5]))
    assert np.all(e == 0) and np.all(v == 0)


# ------------------------------------------------------------------ Hartree
def _gauss_problem(n, order, L=8.0, alpha=1.0, Q=2.0):
    w = make_workload("hydrogen", n=n, order=order)
    mesh = freudenthal_mesh(n, L, order)
    p = KSProblem(order=order, coords=mesh.coords, elems=mesh.elems, dirichlet=mesh.dirichlet,
                  quad=rule_for_order(order), Z=np.array([1.0]), R=np.zeros((1, 3)),
                  occ=np.array([1.0]), L=L, n_H=4, mu=1.0, hartree=True)
    p.setup()
    r2 = np.sum(p.x_q ** 2, axis=-1)
    rho = Q * (alpha / np.pi) ** 1.5 * np.exp(-alpha * r2)
    return p, rho


def _gauss_V(x, alpha=1.0, Q=2.0, c=np.zeros(3)):
    r = np.linalg.norm(x - c, axis=-1)
    return Q * erf(np.sqrt(alpha) * r) / r


@pytest.mark.parametrize("order", [1, 2])
def test_poisson_gaussian_closed_form_converges(order):
    errs = []
    ns = [12, 24] if order == 1 else [6, 12]
    for n in ns:
        p, rho = _gauss_problem(n, order, alpha=0.3)
        wB = _gauss_V(p.coords[p.boundary], alpha=0.3)
        V, it = p.hartree_nodes(rho, wB, tol=1e-13)
        Vq = p.at_quad(V)
        ex = _gauss_V(p.x_q, alpha=0.3)
        errs.append(np.sqrt(p.inner(Vq - ex, Vq - ex)))
    rate = np.log2(errs[0] / errs[1])
    # L2 error O(h^2) for P1 and O(h^3) for P2
    assert rate > (1.8 if order == 1 else 2.7), (errs, rate)


def test_multipole_monopole_exact_for_spherical_density():
    """An isotropic second moment q = s I makes the quadrupole term vanish,
    leaving the monopole Q/|d| exactly; the discrete moments of a centred
    Gaussian approach (Q, 0, Q/(2 alpha) I)."""
    rng = np.random.default_rng(1)
    pts = rng.uniform(-8, 8, size=(40, 3))
    c = np.array([0.1, -0.2, 0.3])
    for f in (0.5, 1.0):
        w = multipole_boundary(pts, 2.0, c, np.zeros(3), 0.7 * np.eye(3), f)
        assert np.allclose(w, 2.0 / np.linalg.norm(pts - c, axis=1), rtol=1e-14)
    p, rho = _gauss_problem(16, 2, L=8.0, alpha=0.3)
    Q, cc, dip, q = density_moments(rho, p.x_q, p.dV)
    assert abs(Q - 2.0) < 1e-5
    assert np.abs(cc).max() < 1e-6 and np.abs(dip).max() < 1e-6
    assert np.allclose(q, 2.0 / (2 * 0.3) * np.eye(3), atol=1e-4)


def test_multipole_half_factor_beats_literal_for_two_gaussians():
    """Two displaced Gaussians have a closed-form potential; the Taylor-correct
    quadrupole (factor 1/2) reproduces it on the boundary better than the
    factor-free print and better than monopole + dipole alone."""
    L = 10.0
    pts = np.array([[L, y, z] for y in np.linspace(-L, L, 7) for z in np.linspace(-L, L, 7)])
    a1, a2 = np.array([1.5, 0.3, 0.0]), np.array([-1.0, -0.2, 0.4])
    alpha = 3.0
    # moments of sum of Gaussians with charges 1 and 2, computed analytically
    Qs = np.array([1.0, 2.0])
    cs = np.array([a1, a2])
    Q = Qs.sum()
    c = (Qs[:, None] * cs).sum(0) / Q
    sig2 = 1.0 / (2 * alpha)
    q = sum(Qk * (np.outer(ck - c, ck - c) + sig2 * np.eye(3)) for Qk, ck in zip(Qs, cs))
    exact = sum(_gauss_V(pts, alpha, Qk, ck) for Qk, ck in zip(Qs, cs))
    e_half = np.abs(multipole_boundary(pts, Q, c, np.zeros(3), q, 0.5) - exact).max()
    e_one = np.abs(multipole_boundary(pts, Q, c, np.zeros(3), q, 1.0) - exact).max()
    e_none = np.abs(multipole_boundary(pts, Q, c, np.zeros(3), q, 0.0) - exact).max()
    assert e_half < 0.2 * e_none and e_half < 0.2 * e_one


# ------------------------------------------------------- coarse interpolation
def test_coarse_interpolation_reproduces_linears_and_partition_of_unity():
    rng = np.random.default_rng(0)
    L, nH = 5.0, 4
    h = 2 * L / nH
    x = rng.uniform(-L + h, L - h, size=(300, 3))     # all coarse vertices interior
    P = coarse_interpolation(x, L, nH)
    ni = nH - 1
    g = -L + h * (1 + np.arange(ni))
    cz, cy, cx = np.meshgrid(g, g, g, indexing="ij")
    cpos = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], 1)
    assert np.allclose(P.sum(1), 1.0, atol=1e-14)
    assert np.allclose(P @ cpos, x, atol=1e-13)
    assert np.all(P >= -1e-15) and np.all((P > 0).sum(1) <= 4)


def test_nested_meshes_give_coarse_galerkin_matrices():
    """Unmoved fine Kuhn mesh with n = 2 n_H refines the coarse Kuhn mesh, so
    P^T K_h P and P^T M_h P equal the matrices assembled on T_H."""
    L, nH = 4.0, 3
    for order in (1, 2):
        pf = KSProblem(order=order, coords=freudenthal_mesh(2 * nH, L, order).coords,
                       elems=freudenthal_mesh(2 * nH, L, order).elems,
                       dirichlet=freudenthal_mesh(2 * nH, L, order).dirichlet,
                       quad=rule_for_order(order), Z=np.array([1.0]), R=np.zeros((1, 3)),
                       occ=np.array([1.0]), L=L, n_H=nH, mu=1.0, hartree=False)
        pf.setup()
        coarse = freudenthal_mesh(nH, L, 1)
        pc = KSProblem(order=1, coords=coarse.coords, elems=coarse.elems,
                       dirichlet=coarse.dirichlet, quad=rule_for_order(1), Z=np.array([1.0]),
                       R=np.zeros((1, 3)), occ=np.array([1.0]), L=L, n_H=nH, mu=1.0,
                       hartree=False)
        pc.setup()
        P = pf.P
        assert np.allclose(P.T @ (pf.K_II @ P), pc.K_II.toarray(), atol=1e-12)
        assert np.allclose(P.T @ (pf.M_II @ P), pc.M_II.toarray(), atol=1e-12)


# ------------------------------------------------------------------ hydrogen
def _hydrogen_lowest(n, order=1, Zc=1.0, scale=1.0, k=1):
    mesh = freudenthal_mesh(n, 10.0 * scale, order)
    p = KSProblem(order=order, coords=mesh.coords, elems=mesh.elems, dirichlet=mesh.dirichlet,
                  quad=rule_for_order(order), Z=np.array([Zc]), R=np.zeros((1, 3)),
                  occ=np.ones(k), L=10.0 * scale, n_H=4, mu=8.0, hartree=False, xc_mode="none")
    p.setup()
    A = p.A_linear()
    vals = sla.eigsh(A, k=k, M=p.M_II, sigma=-0.6 * Zc * Zc, which="LM",
                     return_eigenvectors=False)
    return np.sort(vals)


def test_hydrogen_eigenvalue_converges_to_minus_half():
    """Closed form: the 1s level of -1/2 Laplace - 1/r is -1/2 Ha (the box
    truncation error at L = 10 is below 1e-7).  Galerkin eigenvalues converge
    from above; P2 beats P1 on the same node lattice."""
    lam = [_hydrogen_lowest(n)[0] for n in (8, 16, 32)]
    assert lam[0] > lam[1] > lam[2] > -0.5
    err = [l + 0.5 for l in lam]
    assert err[0] / err[1] > 1.6 and err[1] / err[2] > 1.6
    lam_p2 = [_hydrogen_lowest(n, 2)[0] for n in (8, 16)]
    assert lam_p2[0] > lam_p2[1] > -0.5
    assert lam_p2[0] < lam[1] and lam_p2[1] < lam[2]     # same nodes, better value
    assert (lam_p2[0] + 0.5) / (lam_p2[1] + 0.5) > 2.5
    assert abs(lam_p2[1] + 0.5) < 0.04


def test_hydrogen_exact_charge_scaling():
    """Mesh scaled by 1/Z with nuclear charge Z gives lambda = Z^2 lambda(1)."""
    l1 = _hydrogen_lowest(6)[0]
    l3 = _hydrogen_lowest(6, Zc=3.0, scale=1.0 / 3.0)[0]
    assert abs(l3 - 9.0 * l1) < 1e-11 * abs(l3)


def test_external_potential_is_coulomb():
    x = np.array([[0.0, 1.0, 0.0], [0.0, 2.0, 0.0]])
    v = external_potential(x, np.array([2.0, 1.0]), np.array([[0, 0, 0], [1.0, 0, 0]]))
    assert abs(v[0] - (-2.0 - 1.0 / np.sqrt(2.0))) < 1e-15
    assert abs(v[1] - (-1.0 - 1.0 / np.sqrt(5.0))) < 1e-15


# ---------------------------------------------------------------- solvers
def test_jacobi_pcg_residual_recomputed():
    p = KSProblem.from_workload(make_workload("hydrogen", n=8))
    S = (p.A_linear() + p.mu * p.M_II).tocsr()
    rng = np.random.default_rng(3)
    B = rng.normal(size=(p.N, 3))
    X, it, rr = jacobi_pcg(S, B, None, tol=1e-10)
    true = np.linalg.norm(B - S @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(true < 2e-10) and np.all(it > 0)
    Xd = np.linalg.solve(S.toarray(), B)
    assert np.abs(X - Xd).max() < 1e-8 * np.abs(Xd).max()
