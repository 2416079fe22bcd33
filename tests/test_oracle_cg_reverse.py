"""Pins for the oracle's reverse mode through the truncated Jacobi-PCG of the
block BVP solve (eq. Aux_Linear_Problem), against things it does not share:

* central finite differences of L = sum(Xbar * X_K) in the quadrature
  potential V and in B, for the tolerance-stopped solve and for a fixed
  iteration count (every column truncated early);
* a block's gradient is the sum of its columns' (the columns only share S);
* for a converged solve it tends to the implicit adjoint of the exact
  solution, -Y X^T with S Y = Xbar.
"""
import numpy as np
import pytest

from ks_inputs import make_workload
from oracle.step import KSProblem
from oracle.cg_reverse import truncated_pcg, truncated_pcg_vjp, potential_gradient


def _setup(k=3, n=4, seed=1):
    w = make_workload("small_molecule", n=n, order=1, k=k)
    p = KSProblem.from_workload(w, mu=4.0)
    rng = np.random.default_rng(seed)
    V0 = p.vext_q + 0.3 * rng.standard_normal(p.vext_q.shape)
    A0 = (0.5 * p.K_II + p.mu * p.M_II).tocsr()
    S = lambda V: (A0 + p.potential_matrix(V)).tocsr()
    B = rng.standard_normal((p.N, k))
    X0 = 0.1 * rng.standard_normal((p.N, k))
    Xbar = rng.standard_normal((p.N, k))
    return p, S, V0, B, X0, Xbar, rng


@pytest.mark.parametrize("tol,max_it", [(1e-7, 500), (0.0, 6)])
def test_gradient_matches_finite_differences(tol, max_it):
    p, S, V0, B, X0, Xbar, rng = _setup()
    Sbar, Bbar = truncated_pcg_vjp(S(V0), B, X0, tol, max_it, Xbar)
    g = potential_gradient(p, Sbar)
    _, its, _ = truncated_pcg(S(V0), B, X0, tol, max_it)
    assert its.min() > 3
    L = lambda V, Bm: float(np.sum(Xbar * truncated_pcg(S(V), Bm, X0, tol, max_it)[0]))
    h = 1e-6
    dV = rng.standard_normal(V0.shape)
    fd = (L(V0 + h * dV, B) - L(V0 - h * dV, B)) / (2 * h)
    assert abs(fd - np.sum(g * dV)) < 1e-6 * abs(fd)
    dB = rng.standard_normal(B.shape)
    fdb = (L(V0, B + h * dB) - L(V0, B - h * dB)) / (2 * h)
    assert abs(fdb - np.sum(Bbar * dB)) < 1e-6 * abs(fdb)


def test_block_gradient_is_the_sum_of_column_gradients():
    p, S, V0, B, X0, Xbar, _ = _setup(k=3)
    Sbar, Bbar = truncated_pcg_vjp(S(V0), B, X0, 1e-7, 500, Xbar)
    tot = np.zeros_like(Sbar)
    for c in range(3):
        Sc, Bc = truncated_pcg_vjp(S(V0), B[:, [c]], X0[:, [c]], 1e-7, 500, Xbar[:, [c]])
        tot += Sc
        assert np.allclose(Bc[:, 0], Bbar[:, c], rtol=1e-10, atol=1e-13)
    assert np.abs(tot - Sbar).max() < 1e-10 * np.abs(Sbar).max()


def test_converged_solve_tends_to_the_implicit_adjoint():
    p, S, V0, B, X0, Xbar, _ = _setup(k=2)
    S0 = S(V0)
    Sbar, Bbar = truncated_pcg_vjp(S0, B, X0, 1e-13, 2000, Xbar)
    Sd = S0.toarray()
    X = np.linalg.solve(Sd, B)
    Y = np.linalg.solve(Sd, Xbar)
    g = potential_gradient(p, Sbar)
    g_imp = potential_gradient(p, -Y @ X.T)
    assert np.abs(g - g_imp).max() < 1e-8 * np.abs(g_imp).max()
    assert np.abs(Bbar - Y).max() < 1e-8 * np.abs(Y).max()
