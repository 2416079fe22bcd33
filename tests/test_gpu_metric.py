"""The mesh-moving calls of Algorithm 2 on the GPU against the oracle:
ks_mesh_metric (the Hessian metric of sqrt(rho), eqs. m1-m2), ks_move_nodes
(the metric spring mover, including the step-halving path) and
ks_interpolate_field (Algorithm 1 for nodal fields).  The oracle's metric is
the mover's input on both sides."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from ks_inputs import make_workload
from ks_inputs.mesh import freudenthal_mesh
from oracle.coarse import interpolation_in_mesh
from oracle.metric import nodal_sqrt_density, recover_hessian, metric_from_hessian, move_nodes as o_move

DEV = "cuda:0"
SIX = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def _six(M):
    return np.stack([M[:, i, j] for i, j in SIX], axis=1)


def _full(M6):
    M = np.empty((M6.shape[0], 3, 3))
    for c, (i, j) in enumerate(SIX):
        M[:, i, j] = M[:, j, i] = M6[:, c]
    return M


@pytest.mark.parametrize("name,n,eps", [("lih", 8, 1e-2), ("ch4", 7, 3e-3)])
def test_metric_matches_oracle(name, n, eps):
    from paper_2404_19249_amd import mesh_metric
    w = make_workload(name, n=n)
    m = w.mesh
    print(f"[case] metric {name} n={n} eps={eps}", flush=True)
    rng = np.random.default_rng(21)
    N = int((m.dirichlet == 0).sum())
    psi = rng.standard_normal((N, w.k)) * np.exp(-np.linalg.norm(m.coords[m.dirichlet == 0], axis=1))[:, None]
    h_min, h_max = 0.05, 4.0
    ref = _six(metric_from_hessian(recover_hessian(m.coords, m.elems, nodal_sqrt_density(
        m.n_nodes, m.dirichlet, psi, w.occ)), eps, h_min, h_max))
    got = mesh_metric(m, torch.tensor(psi, device=DEV), w.occ, eps, h_min, h_max).cpu().numpy()
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert np.abs(got - ref).max() / np.abs(ref).max() < 1e-10
    assert (np.abs(got - ref) / scale).max() < 1e-9
    # every metric is positive definite with eigenvalues inside the clamp
    lam = np.linalg.eigvalsh(_full(got))
    assert lam.min() >= (1.0 / h_max ** 2) * (1 - 1e-9) and lam.max() <= (1.0 / h_min ** 2) * (1 + 1e-9)


@pytest.mark.parametrize("omega,amp,sweeps", [(0.5, 50.0, 3), (1.9, 1e3, 3)])
def test_mover_matches_oracle(omega, amp, sweeps):
    from paper_2404_19249_amd import move_nodes
    m = freudenthal_mesh(8, 1.0, 1)
    x0 = m.coords
    print(f"[case] mover omega={omega} amp={amp}", flush=True)
    # an anisotropic metric, larger near the origin
    base = np.diag([1.0, 2.0, 0.5])
    M = (1.0 + amp * np.exp(-(x0 ** 2).sum(1) / 0.05))[:, None, None] * base
    x_ref, hv_ref = o_move(x0, m.elems, M, m.dirichlet, omega=omega, sweeps=sweeps)
    x, hv = move_nodes(m, torch.tensor(_six(M), device=DEV), omega=omega, sweeps=sweeps)
    assert hv == hv_ref
    assert np.abs(x - x_ref).max() < 1e-12
    assert np.array_equal(x[m.dirichlet == 1], x0[m.dirichlet == 1])


def test_interpolate_field_matches_oracle():
    from paper_2404_19249_amd import interpolate_field
    src = make_workload("lih", n=6).mesh
    dst = make_workload("lih", n=9).mesh
    rng = np.random.default_rng(5)
    F = rng.standard_normal((src.n_nodes, 6))
    P = interpolation_in_mesh(dst.coords, src.coords, src.elems, np.zeros(src.n_nodes, dtype=np.uint8))
    got = interpolate_field(src, torch.tensor(F, device=DEV), dst.coords).cpu().numpy()
    # the two sides take barycentric coordinates by different formulas
    # (Cramer's rule against an inverse Jacobian) on coordinates up to 10
    assert np.abs(got - P @ F).max() < 1e-11 * np.abs(F).max()


def test_mesh_calls_reject_bad_input():
    from paper_2404_19249_amd import move_nodes, mesh_metric, KSError
    m2 = make_workload("lih", n=3, order=2).mesh
    with pytest.raises(KSError):
        mesh_metric(m2, torch.zeros(10, 2, dtype=torch.float64, device=DEV), [2.0, 2.0], 1e-2, 0.1, 1.0)
    m = freudenthal_mesh(4, 1.0, 1)
    M = torch.zeros(m.n_nodes, 6, dtype=torch.float64, device=DEV)
    M[:, :3] = 1.0
    with pytest.raises(KSError):
        move_nodes(m, M, omega=2.5)
