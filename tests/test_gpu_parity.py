"""Parity of the HIP path with the CPU oracle, call by call through the C ABI.

Tolerances: 1e-10 relative for FP64 quantities (both sides solve iterative
sub-problems to 1e-13 so truncation stays far below that); 1e-8 Ha for the
mixed-precision eigenvalues."""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from ks_inputs import make_workload
from oracle.step import KSProblem, ks_scf_step, initial_guess, small_eig
from oracle.xc import lda_xc

TIGHT = dict(tol_solve=1e-13, tol_inner=1e-11, tol_poisson=1e-13)
DEV = "cuda:0"


def _ctx(w, **kw):
    from paper_2404_19249_amd import KSContext
    args = dict(TIGHT)
    args.update(kw)
    print(f"[case] {w.name} order={w.mesh.order} n={w.mesh.n} k={w.k}", flush=True)
    return KSContext.from_workload(w, **args)


def _csr(ctx, which):
    rp, cl, vl = ctx.export_operator(which)
    return sp.csr_matrix((vl, cl, rp), shape=(ctx.N, ctx.N))


def _rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = [("hydrogen", dict(n=6)), ("small_molecule", dict(n=4)),
         ("small_molecule", dict(n=5, order=1)), ("mixed", dict(n=5, k=6))]


@pytest.mark.parametrize("name,kw", CASES)
def test_static_operators_match_oracle(name, kw):
    w = make_workload(name, **kw)
    ctx = _ctx(w)
    p = KSProblem.from_workload(w)
    assert ctx.N == p.N and ctx.nnz == p.K_II.nnz
    assert abs(ctx.mu - p.mu) < 1e-12 * p.mu
    for which, ref in [(1, p.K_II), (2, p.M_II), (3, p.A_linear())]:
        A = _csr(ctx, which)
        d = (A - ref).tocsr()
        assert np.abs(d.data).max(initial=0) < 1e-12 * np.abs(ref.data).max(), which


@pytest.mark.parametrize("name,kw", CASES[1:])
def test_assembled_hamiltonian_matches_oracle(name, kw):
    w = make_workload(name, **kw)
    ctx = _ctx(w)
    p = KSProblem.from_workload(w)
    th, Psi = initial_guess(p, w.k)
    psi = torch.tensor(Psi, device=DEV)
    out = ctx.assemble(psi, w.occ)
    rho = p.density(Psi)
    assert _rel(out["rho_q"].cpu().numpy(), rho) < 1e-12
    wB = p.boundary_data(rho)
    VH, _ = p.hartree_nodes(rho, wB, 1e-14)
    assert _rel(out["vh_nodes"].cpu().numpy(), VH) < 1e-10
    _, vxc = lda_xc(rho, p.xc_mode)
    veff = p.vext_q + p.at_quad(VH) + vxc
    assert _rel(out["veff_q"].cpu().numpy(), veff) < 1e-10
    S_ref = (0.5 * p.K_II + p.potential_matrix(veff) + p.mu * p.M_II).tocsr()
    d = (_csr(ctx, 0) - S_ref).tocsr()
    assert np.abs(d.data).max(initial=0) < 1e-11 * np.abs(S_ref.data).max()
    e = out["energies"]
    assert abs(e["E_H"] - 0.5 * p.inner(p.at_quad(VH), rho)) < 1e-10 * abs(e["E_H"])


@pytest.mark.parametrize("name,kw", CASES)
def test_block_solve_matches_oracle(name, kw):
    w = make_workload(name, **kw)
    ctx = _ctx(w)
    p = KSProblem.from_workload(w)
    th, Psi = initial_guess(p, w.k)
    psi = torch.tensor(Psi, device=DEV)
    ctx.assemble(psi, w.occ, want_fields=False)
    hat, st = ctx.block_solve(psi, th)
    assert st["converged"]
    # oracle solve of the same system
    from oracle.step import block_solve
    rho = p.density(Psi)
    if p.hartree or p.xc_mode != "none":
        VH, _ = p.hartree_nodes(rho, p.boundary_data(rho), 1e-14)
        _, vxc = lda_xc(rho, p.xc_mode)
        veff = p.vext_q + p.at_quad(VH) + vxc
    else:
        veff = p.vext_q
    S = (0.5 * p.K_II + p.potential_matrix(veff) + p.mu * p.M_II).tocsr()
    ref, its, rr = block_solve(p, S, Psi, th, tol=1e-13)
    assert _rel(hat.cpu().numpy(), ref) < 1e-10
    assert max(st["relres"]) < 1e-12
    # the iteration counts follow the same recurrence
    assert np.abs(np.array(st["iters"]) - its).max() <= 2


@pytest.mark.parametrize("name,kw", CASES[:2])
def test_projection_matches_oracle(name, kw):
    w = make_workload(name, **kw)
    ctx = _ctx(w)
    p = KSProblem.from_workload(w)
    rng = np.random.default_rng(7)
    hat = rng.normal(size=(p.N, w.k))
    ht = torch.tensor(hat, device=DEV)
    G = p.P.T @ (p.M_II @ p.P)
    T = np.linalg.solve(G, p.P.T @ (p.M_II @ hat))
    Z = np.hstack([p.P, hat - p.P @ T])
    for which, H in [(0, p.M_II), (1, p.A_linear())]:
        F = ctx.augmented_project(ht, which).cpu().numpy()
        ref = Z.T @ (H @ Z)
        assert _rel(F, ref) < 1e-11, which


def test_small_eigensolver_matches_dense_reference():
    w = make_workload("hydrogen", n=6)
    ctx = _ctx(w, k_max=8)
    rng = np.random.default_rng(3)
    for m, k in [(12, 3), (35, 8), (31, 1)]:
        X = rng.normal(size=(200, m))
        Mm = np.diag(rng.uniform(1, 2, 200))
        Am = rng.normal(size=(200, 200)); Am = Am + Am.T
        FA, FB = X.T @ Am @ X, X.T @ Mm @ X
        U, lam, rank = ctx.small_eig(torch.tensor(FA, device=DEV), torch.tensor(FB, device=DEV), k)
        th, Uref, r2, _ = small_eig(FA, FB, k)
        assert rank == r2 == m
        assert _rel(lam, th) < 1e-11
        assert _rel(U.cpu().numpy(), Uref) < 1e-8


@pytest.mark.parametrize("name,kw", CASES)
def test_initial_guess_matches_oracle(name, kw):
    w = make_workload(name, **kw)
    ctx = _ctx(w)
    p = KSProblem.from_workload(w)
    psi, lam = ctx.initial_guess(w.k)
    th, Psi = initial_guess(p, w.k)
    assert _rel(lam, th) < 1e-11
    assert _rel(psi.cpu().numpy(), Psi) < 1e-8


def test_hydrogen_steps_match_oracle_full_size():
    """Hydrogen-like workload at full size (16^3 P1, k = 1, 3 steps)."""
    w = make_workload("hydrogen")
    ctx = _ctx(w)
    p = KSProblem.from_workload(w)
    th, Psi = initial_guess(p, 1)
    psi = torch.tensor(Psi, device=DEV)
    lam = th.copy()
    for step in range(3):
        lam, rep = ctx.scf_step(psi, lam, w.occ)
        r = ks_scf_step(p, Psi, th, tol_solve=1e-13, want_eks=False)
        Psi, th = r.Psi, r.lam
        assert _rel(lam, th) < 1e-10, step
        assert _rel(psi.cpu().numpy(), Psi) < 1e-8
        assert abs(rep["E_total"] - r.energies["total"]) < 1e-10 * abs(r.energies["total"])
    assert -0.5 < lam[0] < -0.3


@pytest.mark.parametrize("name,kw", CASES[1:])
def test_nonlinear_step_matches_oracle(name, kw):
    w = make_workload(name, **kw)
    ctx = _ctx(w)
    p = KSProblem.from_workload(w)
    th, Psi = initial_guess(p, w.k)
    psi = torch.tensor(Psi, device=DEV)
    rho = torch.empty(ctx.n_elems, ctx.n_q, dtype=torch.float64, device=DEV)
    lam, rep = ctx.scf_step(psi, th, w.occ, rho_out=rho)
    r = ks_scf_step(p, Psi, th, tol_solve=1e-13, tol_inner=1e-11, tol_poisson=1e-13,
                    want_eks=False)
    assert rep["res_inner"] < 1e-11
    assert _rel(lam, r.lam) < 1e-10
    assert abs(rep["E_total"] - r.energies["total"]) < 1e-10 * abs(r.energies["total"])
    d = rho.cpu().numpy() - r.rho_q
    assert np.sqrt(p.inner(d, d)) < 1e-9 * np.sqrt(p.inner(r.rho_q, r.rho_q))
    # orbitals up to sign (fixed by the largest coefficient) and degeneracy
    G = psi.cpu().numpy().T @ (p.M_II @ r.Psi)
    assert np.abs(np.abs(np.diag(G)) - 1).max() < 1e-8


def test_mixed_precision_solve_reaches_fp64_accuracy():
    w = make_workload("small_molecule", n=6)
    ctx = _ctx(w, tol_solve=1e-8)
    p = KSProblem.from_workload(w)
    th, Psi = initial_guess(p, w.k)
    psi = torch.tensor(Psi, device=DEV)
    ctx.assemble(psi, w.occ, want_fields=False)
    h64, s64 = ctx.block_solve(psi, th, "fp64")
    h32, s32 = ctx.block_solve(psi, th, "mixed")
    assert s32["converged"] and max(s32["relres"]) < 1e-8
    assert s32["refinements"] >= 2
    d = (h32 - h64).abs().max().item() / h64.abs().max().item()
    assert d < 1e-6


# The solve tolerance the benchmark times.  The eigenvalues of one step move
# to first order with the BVP solution error, with a coefficient set by the
# eigen-residual of the step's input: on the bench workload, from the state
# after one step, 1.8e-8 Ha at a 1e-8 relative residual and 2.3e-9 Ha at
# 1e-9; from the coarse Ritz guess itself the coefficient is about 15 times
# larger.  The timed solves run to 1e-9, inside the metric's 1e-8 bound, and
# every timed step starts from the state after one step.
BENCH_TOL_SOLVE = 1e-9


@pytest.mark.parametrize("name,kw", [("small_molecule", dict(n=6)), ("mixed", dict(n=5, k=6))])
@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_step_at_bench_tolerance_matches_tight_oracle_step(name, kw, prec):
    """One step with the BVPs solved to the benchmark's tolerance, in the
    FP32-in-FP64 refinement form and in FP64, against the oracle's step
    with tightly solved sub-problems, both from the oracle's state after one
    step from the coarse Ritz guess (the benchmark's timed input is such a
    state): every eigenvalue within 1e-8 Ha, and E_total within
    sum_i f_i 1e-8 Ha."""
    w = make_workload(name, **kw)
    p = KSProblem.from_workload(w)
    th0, Psi0 = initial_guess(p, w.k)
    tight = dict(tol_solve=1e-13, tol_inner=1e-11, tol_poisson=1e-13, want_eks=False)
    s1 = ks_scf_step(p, Psi0, th0, **tight)
    Psi, th = s1.Psi, s1.lam
    ref = ks_scf_step(p, Psi, th, **tight)
    ctx = _ctx(w, tol_solve=BENCH_TOL_SOLVE, tol_inner=1e-11, tol_poisson=1e-12)
    psi = torch.tensor(Psi, device=DEV)
    lam, rep = ctx.scf_step(psi, th, w.occ, precision=prec)
    assert rep["status"] == 0 and rep["solve"]["converged"]
    assert max(rep["solve"]["relres"]) <= BENCH_TOL_SOLVE
    if prec == "mixed":
        assert rep["solve"]["refinements"] >= 2
    err = np.abs(lam - ref.lam).max()
    e_err = abs(rep["E_total"] - ref.energies["total"])
    print(f"{name} {prec}: eig err {err:.2e} Ha, E_total err {e_err:.2e} Ha")
    assert err < 1e-8
    assert e_err < 1e-8 * float(np.sum(w.occ))
    ctx.close()


def _direct_dense_scf(p, k, tol=1e-12, beta=0.5, max_it=400):
    """Self-consistent field on the whole fine space with dense eigensolves
    (scipy as an independent checking tool): the fixed point a converged run
    of Algorithm 3 must reach."""
    import scipy.linalg as sla
    A0 = (0.5 * p.K_II + p.Mext_II).toarray()
    Md = p.M_II.toarray()
    lam, V = sla.eigh(A0, Md)
    rho = p.density(V[:, :k])
    for _ in range(max_it):
        wB = p.boundary_data(rho)
        VH, _ = p.hartree_nodes(rho, wB, 1e-14)
        _, vxc = lda_xc(rho, p.xc_mode)
        A = A0 + p.potential_matrix(p.at_quad(VH) + vxc).toarray()
        lam, V = sla.eigh(A, Md)
        rho_out = p.density(V[:, :k])
        d = rho_out - rho
        if np.sqrt(p.inner(d, d)) < tol:
            return lam[:k], rho_out
        rho = rho + beta * d
    raise RuntimeError("direct SCF did not converge")


def test_outer_loop_reaches_direct_scf():
    """Algorithm 3 run to convergence on the GPU (ks_scf_run) reaches the
    direct dense SCF on the fine space (the fixed point of the augmented
    iteration), and the two energy expressions coincide there."""
    w = make_workload("small_molecule", n=6, order=1, k=2)
    w.n_H = 4
    p = KSProblem.from_workload(w, mu=4.0)
    lam_d, rho_d = _direct_dense_scf(p, 2)
    ctx = _ctx(w, mu=4.0, k_max=2)
    th, Psi = initial_guess(p, 2)
    psi = torch.tensor(Psi, device=DEV)
    rho = torch.empty(ctx.n_elems, ctx.n_q, dtype=torch.float64, device=DEV)
    lam, rep = ctx.scf_run(psi, th, w.occ, tol=1e-10, max_steps=300, rho_out=rho)
    print(rep, lam, lam_d)
    assert rep["converged"] and rep["res_outer"] < 1e-10
    assert np.abs(lam - lam_d).max() < 1e-8
    d = rho.cpu().numpy() - rho_d
    assert np.sqrt(p.inner(d, d)) < 1e-8
    assert abs(rep["E_total"] - rep["E_KS"]) < 1e-8
    # the reported density change is the quadrature norm of the last step's
    lam2, rep2 = ctx.scf_step(psi, lam, w.occ, rho_out=rho)
    assert rep2["res_outer"] < 1e-10


def test_nonnested_coarse_space_matches_oracle():
    """Sec. 3.2 with a coarse mesh that is not nested in the fine one: the
    coarse Gram block P^T M P of the GPU's I_H^h (Algorithm 1: bucket-grid
    nearest vertex and barycentric walk) equals the oracle's, whose P comes
    from the by-definition location; one nonlinear step on that augmented
    space matches the oracle step."""
    from ks_inputs import jittered_coarse_mesh
    w = make_workload("small_molecule", n=5)
    cm = jittered_coarse_mesh(4, w.mesh.L, amp=0.3, seed=7)
    ctx = _ctx(w, coarse=cm)
    p = KSProblem.from_workload(w, coarse=cm)
    nH = p.P.shape[1]
    assert ctx.N_H == nH
    G = ctx.debug_buffer("GPP", nH * nH).cpu().numpy().reshape(nH, nH)
    G_ref = p.P.T @ (p.M_II @ p.P)
    assert _rel(G, G_ref) < 1e-12
    th, Psi = initial_guess(p, w.k)
    psi = torch.tensor(Psi, device=DEV)
    lam, rep = ctx.scf_step(psi, th, w.occ)
    r = ks_scf_step(p, Psi, th, tol_solve=1e-13, tol_inner=1e-11, tol_poisson=1e-13, want_eks=False)
    assert _rel(lam, r.lam) < 1e-10
    assert abs(rep["E_total"] - r.energies["total"]) < 1e-10 * abs(r.energies["total"])


def test_inner_iteration_cap_matches_oracle_and_blocks_backward():
    """An inner iteration stopped at its limit: the step reports
    KS_NOT_CONVERGED, its eigenvalues, orbitals and E_total equal the
    oracle's step stopped at the same limit (no mixing after the last pass,
    so E_total pairs rho_in with its own potentials), and the adjoint,
    which needs the converged inner fixed point, is refused."""
    from paper_2404_19249_amd import KSError
    w = make_workload("small_molecule", n=4)
    ctx = _ctx(w, max_it_inner=3, tol_inner=1e-14)
    p = KSProblem.from_workload(w)
    th, Psi = initial_guess(p, w.k)
    psi = torch.tensor(Psi, device=DEV)
    lam, rep = ctx.scf_step(psi, th, w.occ)
    r = ks_scf_step(p, Psi, th, tol_solve=1e-13, tol_inner=1e-14, tol_poisson=1e-13,
                    max_inner=3, want_eks=False)
    assert rep["status"] == 1 and rep["inner_iters"] == 3 == r.inner_iters
    assert abs(rep["res_inner"] - r.extra["res_inner"]) < 1e-8 * r.extra["res_inner"]
    assert _rel(lam, r.lam) < 1e-10
    assert abs(rep["E_total"] - r.energies["total"]) < 1e-10 * abs(r.energies["total"])
    assert abs(rep["E_H"] - r.energies["H_in"]) < 1e-10 * abs(r.energies["H_in"])
    with pytest.raises(KSError) as e:
        ctx.step_backward()
    assert e.value.code == -7
    ctx.close()


@pytest.mark.parametrize("name,kw", CASES[:2])
def test_block_cg_matches_oracle(name, kw):
    """KS_PREC_FP64_BLOCK_CG (O'Leary's block CG, one Krylov block for all
    columns) solves the same BVPs as the oracle's per-column PCG; its block
    Krylov space holds every column's own, so it needs no more iterations
    than the slowest column of the per-column recurrence (up to rounding)."""
    w = make_workload(name, **kw)
    ctx = _ctx(w)
    p = KSProblem.from_workload(w)
    th, Psi = initial_guess(p, w.k)
    psi = torch.tensor(Psi, device=DEV)
    ctx.assemble(psi, w.occ, want_fields=False)
    hat, st = ctx.block_solve(psi, th, precision="block_cg")
    _, st_col = ctx.block_solve(psi, th, precision="fp64")
    assert st["converged"]
    from oracle.step import block_solve
    rho = p.density(Psi)
    veff = p.vext_q
    if p.hartree or p.xc_mode != "none":
        VH, _ = p.hartree_nodes(rho, p.boundary_data(rho), 1e-14)
        _, vxc = lda_xc(rho, p.xc_mode)
        veff = p.vext_q + p.at_quad(VH) + vxc
    S = (0.5 * p.K_II + p.potential_matrix(veff) + p.mu * p.M_II).tocsr()
    ref, its, rr = block_solve(p, S, Psi, th, tol=1e-13)
    assert _rel(hat.cpu().numpy(), ref) < 1e-10
    assert max(st["relres"]) < 1e-12
    assert max(st["iters"]) <= max(st_col["iters"]) + 1


def test_block_cg_with_one_column_is_pcg():
    """With k = 1 the block recurrence is the scalar Jacobi-PCG recurrence."""
    w = make_workload("small_molecule", n=6, k=1)
    ctx = _ctx(w)
    psi, lam = ctx.initial_guess(1)
    ctx.assemble(psi, w.occ, want_fields=False)
    a, st_a = ctx.block_solve(psi, lam, precision="block_cg")
    b, st_b = ctx.block_solve(psi, lam, precision="fp64")
    assert abs(st_a["iters"][0] - st_b["iters"][0]) <= 1
    assert _rel(a.cpu().numpy(), b.cpu().numpy()) < 1e-11
