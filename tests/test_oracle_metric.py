"""Pins for the oracle's Hessian metric (Sec. 3.2, eqs. m1-m2) and its
metric spring node mover (the stand-in for the remesher of Algorithm 2).

* gradient recovery reproduces the gradient of a linear function at every
  node of an irregular mesh;
* on a uniform Kuhn mesh the recovered gradient of a quadratic is exact at
  every node off the boundary and the recovered Hessian exact at every node
  two layers in (the vertex patches are point symmetric);
* the metric applies the clamp of eq. m2 to each eigenvalue (all three
  branches checked by hand) and rotates with the Hessian;
* a constant metric, isotropic or not, leaves a uniform mesh where it is;
* a metric peaked at a point draws nodes toward it, lowers the spring energy
  every damped sweep, keeps the Dirichlet nodes and every element valid;
* an over-relaxed sweep that would invert an element is halved instead.
"""
import numpy as np
import pytest

from ks_inputs.mesh import freudenthal_mesh, move_nodes_toward_nuclei
from oracle.metric import (C_D3, nodal_sqrt_density, recover_gradient, recover_hessian,
                           metric_from_hessian, mesh_edges, spring_energy, min_det, move_nodes)

A = np.array([[1.0, 0.3, -0.2], [0.3, -2.0, 0.5], [-0.2, 0.5, 0.7]])
BV = np.array([0.1, -0.4, 0.25])


def _quadratic(x):
    return 0.5 * np.einsum("ni,ij,nj->n", x, A, x) + x @ BV + 0.3


def test_gradient_recovery_is_exact_for_linear_functions():
    m = move_nodes_toward_nuclei(freudenthal_mesh(7, 1.0, 1), np.array([[0.1, 0.2, -0.1]]))
    G = recover_gradient(m.coords, m.elems, m.coords @ BV + 1.0)
    assert np.abs(G - BV).max() < 1e-13


def test_recovery_is_exact_for_quadratics_inside_a_uniform_mesh():
    n, L = 8, 1.0
    m = freudenthal_mesh(n, L, 1)
    x = m.coords
    layer = np.rint((L - np.abs(x).max(axis=1)) / (2 * L / n)).astype(int)
    G = recover_gradient(x, m.elems, _quadratic(x))
    H = recover_hessian(x, m.elems, _quadratic(x))
    assert np.abs(G[layer >= 1] - (x[layer >= 1] @ A + BV)).max() < 1e-13
    assert np.abs(H[layer >= 2] - A).max() < 1e-12
    # and not at the boundary layer, where the patches are cut
    assert np.abs(H[layer == 0] - A).max() > 0.1


def test_metric_clamps_each_eigenvalue():
    assert C_D3 == pytest.approx(9.0 / 32.0)
    eps, hmin, hmax = 1e-2, 0.05, 2.0
    # |lambda| = 1e-4 -> 1/h_max^2; 0.5 -> C_d 0.5 / eps; 1e4 -> 1/h_min^2
    H = np.diag([1e-4, -0.5, 1e4])[None]
    M = metric_from_hessian(H, eps, hmin, hmax)[0]
    assert np.allclose(np.diag(M), [1.0 / hmax ** 2, C_D3 * 0.5 / eps, 1.0 / hmin ** 2], rtol=1e-13)
    assert np.abs(M - np.diag(np.diag(M))).max() < 1e-12
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    Hr = np.diag([0.3, -2.0, 40.0])
    Mr = metric_from_hessian((Q @ Hr @ Q.T)[None], eps, hmin, hmax)[0]
    assert np.allclose(Mr, Q @ metric_from_hessian(Hr[None], eps, hmin, hmax)[0] @ Q.T, atol=1e-10)


def test_nodal_sqrt_density():
    dirichlet = np.array([1, 0, 0, 1, 0], dtype=np.uint8)
    psi = np.array([[0.3, -0.1], [0.0, 0.2], [1.0, 0.5]])
    u = nodal_sqrt_density(5, dirichlet, psi, [2.0, 1.0])
    assert np.allclose(u, [0.0, np.sqrt(0.18 + 0.01), np.sqrt(0.04), 0.0, np.sqrt(2.0 + 0.25)])


@pytest.mark.parametrize("Mc", [np.eye(3) * 4.0, np.diag([1.0, 9.0, 0.25])])
def test_constant_metric_is_a_fixed_point(Mc):
    m = freudenthal_mesh(6, 1.0, 1)
    M = np.broadcast_to(Mc, (m.n_nodes, 3, 3)).copy()
    x, hv = move_nodes(m.coords, m.elems, M, m.dirichlet, omega=1.0, sweeps=3)
    assert hv == 0 and np.abs(x - m.coords).max() < 1e-12


def test_peaked_metric_draws_nodes_and_lowers_the_energy():
    m = freudenthal_mesh(8, 1.0, 1)
    x0 = m.coords
    M = (1.0 + 50.0 * np.exp(-(x0 ** 2).sum(1) / 0.1))[:, None, None] * np.eye(3)
    edges = mesh_edges(m.elems)
    x, E = x0, [spring_energy(x0, edges, M)]
    for _ in range(4):
        x, hv = move_nodes(x, m.elems, M, m.dirichlet, omega=0.5, sweeps=1)
        assert hv == 0
        E.append(spring_energy(x, edges, M))
    assert all(b < a for a, b in zip(E, E[1:]))
    assert np.array_equal(x[m.dirichlet == 1], x0[m.dirichlet == 1])
    assert min_det(x, m.elems) > 0.0
    r0, r1 = np.linalg.norm(x0, axis=1), np.linalg.norm(x, axis=1)
    assert (r1 < 0.35).sum() > (r0 < 0.35).sum()


def test_over_relaxed_sweep_is_halved_instead_of_inverting():
    m = freudenthal_mesh(8, 1.0, 1)
    x0 = m.coords
    M = (1.0 + 1e3 * np.exp(-(x0 ** 2).sum(1) / 0.05))[:, None, None] * np.eye(3)
    with pytest.raises(RuntimeError):
        move_nodes(x0, m.elems, M, m.dirichlet, omega=1.9, sweeps=3, max_halvings=0)
    x, hv = move_nodes(x0, m.elems, M, m.dirichlet, omega=1.9, sweeps=3)
    assert hv > 0 and min_det(x, m.elems) > 0.0
