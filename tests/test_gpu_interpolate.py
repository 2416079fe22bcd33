"""ks_interpolate (Algorithm 1 between two meshes, as Algorithm 2 carries the
orbitals to the next mesh) against the oracle's interpolation matrix, which
locates every point by brute force over all source elements."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from ks_inputs import make_workload
from oracle.coarse import interpolation_in_mesh

DEV = "cuda:0"


def _interior_points(mesh):
    return mesh.coords[np.flatnonzero(mesh.dirichlet == 0)]


@pytest.mark.parametrize("name,n_src,n_dst,k", [("lih", 6, 9, 2), ("ch4", 5, 8, 5), ("hydrogen", 7, 4, 1)])
def test_interpolation_matches_oracle(name, n_src, n_dst, k):
    from paper_2404_19249_amd import KSContext
    src = make_workload(name, n=n_src, k=k).mesh
    w = make_workload(name, n=n_dst, k=k)
    print(f"[case] {name} {n_src}->{n_dst} k={k}", flush=True)
    P = interpolation_in_mesh(_interior_points(w.mesh), src.coords, src.elems, src.dirichlet)
    rng = np.random.default_rng(11)
    psi_src = rng.standard_normal((P.shape[1], k))
    ctx = KSContext.from_workload(w, k_max=max(k, 2))
    out = ctx.interpolate(src, torch.tensor(psi_src, device=DEV)).cpu().numpy()
    ctx.close()
    assert np.abs(out - P @ psi_src).max() < 1e-12 * max(1.0, np.abs(psi_src).max())


def test_orthonormalised_interpolation_matches_oracle():
    """With orthonormalize the columns P psi_src are then made M-orthonormal
    in column order: X R^-1 with X^T M X = R^T R, R upper triangular with a
    positive diagonal (unique)."""
    from paper_2404_19249_amd import KSContext
    from oracle.step import KSProblem
    src = make_workload("ch4", n=6).mesh
    w = make_workload("ch4", n=9)
    P = interpolation_in_mesh(_interior_points(w.mesh), src.coords, src.elems, src.dirichlet)
    rng = np.random.default_rng(12)
    psi_src = rng.standard_normal((P.shape[1], w.k))
    M = KSProblem.from_workload(w).M_II
    X = P @ psi_src
    R = np.linalg.cholesky(X.T @ (M @ X)).T
    ref = np.linalg.solve(R.T, X.T).T
    ctx = KSContext.from_workload(w)
    out = ctx.interpolate(src, torch.tensor(psi_src, device=DEV), orthonormalize=True).cpu().numpy()
    ctx.close()
    assert np.abs(out.T @ (M @ out) - np.eye(w.k)).max() < 1e-12
    assert np.abs(out - ref).max() < 1e-10 * np.abs(ref).max()


def test_interpolation_reproduces_linear_functions_inside():
    """A function linear in x, y, z is P1 on every mesh: carried from one mesh
    to another it is reproduced exactly at every point away from the
    boundary layer (where the source carries zero Dirichlet values)."""
    from paper_2404_19249_amd import KSContext
    src = make_workload("lih", n=6).mesh
    w = make_workload("lih", n=10)
    f = lambda x: 0.3 + x[:, 0] - 2.0 * x[:, 1] + 0.5 * x[:, 2]
    inner = np.flatnonzero(src.dirichlet == 0)
    psi_src = np.stack([f(src.coords[inner]), -f(src.coords[inner])], axis=1)
    ctx = KSContext.from_workload(w, k_max=2)
    out = ctx.interpolate(src, torch.tensor(psi_src, device=DEV)).cpu().numpy()
    ctx.close()
    x = _interior_points(w.mesh)
    # points whose source element has no boundary vertex
    P = interpolation_in_mesh(x, src.coords, src.elems, src.dirichlet)
    bnd = src.dirichlet.astype(bool)
    full = np.abs(P.sum(axis=1) - 1.0) < 1e-12
    assert full.sum() > 0.2 * len(x)
    assert np.abs(out[full, 0] - f(x[full])).max() < 1e-11
    assert np.abs(out[:, 1] + out[:, 0]).max() < 1e-12
    assert bnd.any()


def test_interpolation_rejects_a_p2_source():
    from paper_2404_19249_amd import KSContext
    src = make_workload("lih", n=4, order=2).mesh
    w = make_workload("lih", n=5)
    ctx = KSContext.from_workload(w, k_max=2)
    with pytest.raises(RuntimeError):
        ctx.interpolate(src, torch.zeros(10, 2, dtype=torch.float64, device=DEV))
    ctx.close()
