"""GPU paths that the small parity meshes do not reach: a Hartree multigrid
hierarchy of three and four levels, and the one-stage small eigensolver used
when the augmented space has more than 190 directions.  Each is compared
with the CPU oracle through the C ABI."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from ks_inputs import make_workload
from oracle.step import KSProblem, ks_scf_step, initial_guess, small_eig

DEV = "cuda:0"
TIGHT = dict(tol_solve=1e-13, tol_inner=1e-11, tol_poisson=1e-13)


def _ctx(w, **kw):
    from paper_2404_19249_amd import KSContext
    args = dict(TIGHT)
    args.update(kw)
    print(f"[case] {w.name} order={w.mesh.order} n={w.mesh.n} k={w.k} n_H={w.n_H}", flush=True)
    return KSContext.from_workload(w, **args)


def _rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_hartree_multilevel_vcycle_matches_oracle():
    """V_H of the MG-preconditioned CG against the oracle's Jacobi-PCG
    solution of the same Poisson problem with the same multipole boundary
    data (Sec. 3.1, eq. bd), on a P2 mesh of 16^3 hexes whose hierarchy has
    three levels: the fine P2 operator, P1 on the mesh's own vertices
    (nested; smoothed, an intermediate level) and P1 on a uniform lattice of
    8^3 cells (343 unknowns, inverted)."""
    w = make_workload("small_molecule", n=16)
    ctx = _ctx(w)
    assert ctx.mg_levels == 3
    p = KSProblem.from_workload(w)
    th, Psi = initial_guess(p, w.k)
    out = ctx.assemble(torch.tensor(Psi, device=DEV), w.occ)
    rho = p.density(Psi)
    VH, _ = p.hartree_nodes(rho, p.boundary_data(rho), 1e-14)
    assert _rel(out["vh_nodes"].cpu().numpy(), VH) < 1e-10
    e = out["energies"]
    assert abs(e["E_H"] - 0.5 * p.inner(p.at_quad(VH), rho)) < 1e-10 * abs(e["E_H"])
    ctx.close()


def test_one_stage_eigensolver_matches_oracle_beyond_190():
    """m > 190 does not fit the packed LDS eigensolver; the one-stage
    fallback must give the oracle's eigenpairs (eq. st1)."""
    w = make_workload("hydrogen", n=8)
    w.n_H = 7                               # 216 coarse unknowns
    ctx = _ctx(w, k_max=8)
    rng = np.random.default_rng(5)
    for m, k in [(200, 64), (224, 8)]:
        X = rng.normal(size=(400, m))
        Mm = np.diag(rng.uniform(1, 2, 400))
        Am = rng.normal(size=(400, 400)); Am = Am + Am.T
        FA, FB = X.T @ Am @ X, X.T @ Mm @ X
        U, lam, rank = ctx.small_eig(torch.tensor(FA, device=DEV), torch.tensor(FB, device=DEV), k)
        th, Uref, r2, _ = small_eig(FA, FB, k)
        assert rank == r2 == m
        assert _rel(lam, th) < 1e-10
        U = U.cpu().numpy()
        assert _rel(U, Uref) < 1e-8
    ctx.close()


def test_step_with_augmented_space_beyond_190_matches_oracle():
    """A nonlinear step whose augmented space has N_H + k = 216 + 5 = 221
    directions (one-stage eigensolver in every inner iteration) against the
    oracle step."""
    w = make_workload("small_molecule", n=8)
    w.n_H = 7
    ctx = _ctx(w)
    assert ctx.N_H + w.k > 190
    p = KSProblem.from_workload(w)
    th, Psi = initial_guess(p, w.k)
    psi = torch.tensor(Psi, device=DEV)
    lam, rep = ctx.scf_step(psi, th, w.occ)
    r = ks_scf_step(p, Psi, th, want_eks=False, **{k: v for k, v in TIGHT.items()})
    assert rep["status"] == 0 and rep["res_inner"] < 1e-11
    assert rep["rank"] == r.rank
    assert _rel(lam, r.lam) < 1e-10
    assert abs(rep["E_total"] - r.energies["total"]) < 1e-10 * abs(r.energies["total"])
    ctx.close()
