"""Pins for the oracle's adjoint of one step: the gradient of E_KS(Psi^{l+1})
with respect to V_ext at the quadrature points and the nuclear forces agree
with central finite differences of the whole step (inputs held fixed)."""
import numpy as np
import pytest

from ks_inputs import make_workload
from oracle.step import KSProblem, ks_scf_step, initial_guess, step_backward

KW = dict(tol_solve=1e-14, tol_inner=1e-13, tol_poisson=1e-14)


@pytest.fixture(scope="module")
def state():
    w = make_workload("small_molecule", n=5, order=1, k=2)
    w.n_H = 3
    p = KSProblem.from_workload(w, mu=6.0)
    th, Psi = initial_guess(p, 2)
    for _ in range(2):
        r = ks_scf_step(p, Psi, th, tol_solve=1e-13, tol_inner=1e-12, tol_poisson=1e-14)
        Psi, th = r.Psi, r.lam
    r = ks_scf_step(p, Psi, th, **KW)
    g, F, info = step_backward(p, r, tol=1e-14)
    return p, Psi, th, r, g, F


def test_gradient_matches_directional_finite_difference(state):
    p, Psi, th, r, g, F = state
    rng = np.random.default_rng(1)
    for trial in range(2):
        c = rng.uniform(-2, 2, 3)
        dV = np.exp(-np.sum((p.x_q - c) ** 2, -1) / 4.0)
        h = 1e-4
        Ep = ks_scf_step(p.with_external(vext_q=p.vext_q + h * dV), Psi, th, **KW).energies["KS"]
        Em = ks_scf_step(p.with_external(vext_q=p.vext_q - h * dV), Psi, th, **KW).energies["KS"]
        fd = (Ep - Em) / (2 * h)
        adj = np.sum(g * dV)
        assert abs(fd - adj) < 1e-6 * abs(fd)
        # the implicit (BVP) part of the gradient is not negligible here
        hf = np.sum(p.dV * r.rho_q * dV)
        assert abs(hf - fd) > 1e-4 * abs(fd)


def test_forces_match_finite_differences(state):
    p, Psi, th, r, g, F = state
    h = 1e-4
    for a, d in [(0, 2), (1, 0), (2, 1)]:
        Rp = p.R.copy(); Rp[a, d] += h
        Rm = p.R.copy(); Rm[a, d] -= h
        Ep = ks_scf_step(p.with_external(R=Rp), Psi, th, **KW).energies["KS"]
        Em = ks_scf_step(p.with_external(R=Rm), Psi, th, **KW).energies["KS"]
        fd = -(Ep - Em) / (2 * h)
        assert abs(fd - F[a, d]) < 1e-5 * max(1.0, abs(fd)), (a, d, fd, F[a, d])


def test_total_force_of_isolated_molecule_is_small(state):
    """Translation invariance is broken only by the box and the mesh: the net
    force is much smaller than the individual forces."""
    p, Psi, th, r, g, F = state
    assert np.linalg.norm(F.sum(0)) < 0.5 * np.abs(F).max()
