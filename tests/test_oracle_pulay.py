"""Pins for the oracle's derivative of one step's E_KS with respect to the
vertex coordinates (oracle/pulay.py), against things it does not share:

* central finite differences of the oracle's own step energy on moved
  meshes (same inputs Psi^l, lambda^l, boundary data and coarse matrix P),
  for P1 and P2 elements;
* nuclear forces with mesh motion against central differences in which the
  nuclei and the mesh move together;
* invariance of the step under a rigid translation or rotation of mesh and
  nuclei: sum_v dE/dX_v = sum_a F_a and sum_v X_v x dE/dX_v = sum_a R_a x F_a,
  with F the fixed-mesh forces of the oracle's adjoint.

A mistake in any term that does not vanish at the inner fixed point (a
dropped pair, a wrong weight or sign) moves the directional derivative by
1e-3 or more relative; the differences agree to about 1e-8.  The
M-orthogonalisation term vanishes at the fixed point (P^T R = 0), so no pin
can see it."""
import numpy as np
import pytest

from ks_inputs import make_workload
from oracle.step import KSProblem, ks_scf_step, initial_guess, step_backward
from oracle.pulay import step_mesh_gradient, forces_with_mesh_motion, p2_midpoint_field

TIGHT = dict(tol_solve=1e-14, tol_inner=1e-13, tol_poisson=1e-14)


def _setup(order, name="small_molecule"):
    if name == "hydrogen":  # the linear case: no Hartree, no exchange-correlation
        w = make_workload("hydrogen", n=4, order=order, k=1)
    else:
        w = make_workload(name, n=4 if order == 1 else 3, order=order, k=2)
    w.n_H = 3
    p = KSProblem.from_workload(w, mu=6.0)
    th, Psi = initial_guess(p, 2)
    r = ks_scf_step(p, Psi, th, **TIGHT)
    Psi, th = r.Psi, r.lam
    r = ks_scf_step(p, Psi, th, **TIGHT)
    return p, Psi, th, r


def _energy(p, Psi, th, r, coords, R=None):
    q = p.moved(coords)
    if R is not None:
        q = q.with_external(R=R)
    return ks_scf_step(q, Psi, th, w_B=r.extra["w_B"], **TIGHT).energies["KS"]


@pytest.mark.parametrize("order,name", [(1, "small_molecule"), (2, "small_molecule"), (1, "hydrogen")])
def test_mesh_gradient_matches_finite_differences(order, name):
    p, Psi, th, r = _setup(order, name)
    gX = step_mesh_gradient(p, r, Psi, th)
    rng = np.random.default_rng(4)
    D = p2_midpoint_field(p.elems, rng.standard_normal(p.coords.shape))
    h = 1e-5
    fd = (_energy(p, Psi, th, r, p.coords + h * D) - _energy(p, Psi, th, r, p.coords - h * D)) / (2 * h)
    assert abs(fd - np.sum(gX * D)) < 1e-6 * abs(fd)
    # edge nodes carry no derivative: the geometry is that of the vertices
    if order == 2:
        assert np.all(gX[np.unique(p.elems[:, 4:])] == 0.0)


def test_translation_and_rotation_identities():
    p, Psi, th, r = _setup(1)
    gX = step_mesh_gradient(p, r, Psi, th)
    _, F, _ = step_backward(p, r, tol=1e-14)
    scale = np.abs(F).max()
    assert np.abs(gX.sum(axis=0) - F.sum(axis=0)).max() < 1e-9 * scale
    tq = np.cross(p.coords, gX).sum(axis=0) - np.cross(p.R, F).sum(axis=0)
    assert np.abs(tq).max() < 1e-9 * scale * np.abs(p.coords).max()


def test_forces_with_mesh_motion_match_finite_differences():
    p, Psi, th, r = _setup(1)
    gX = step_mesh_gradient(p, r, Psi, th)
    _, F, _ = step_backward(p, r, tol=1e-14)
    # nodes follow the nearest nuclei with Gaussian weights
    d2 = np.sum((p.coords[:, None, :] - p.R[None, :, :]) ** 2, axis=-1)
    Wm = np.exp(-d2 / 4.0)
    Fm = forces_with_mesh_motion(F, gX, Wm)
    h = 1e-5
    for a, d in [(0, 0), (1, 2), (2, 1)]:
        E = []
        for s in (1, -1):
            R = p.R.copy()
            R[a, d] += s * h
            X = p.coords.copy()
            X[:, d] += s * h * Wm[:, a]
            E.append(_energy(p, Psi, th, r, X, R))
        fd = -(E[0] - E[1]) / (2 * h)
        assert abs(fd - Fm[a, d]) < 1e-6 * np.abs(Fm).max()
        # the mesh term is not negligible
        assert abs(Fm[a, d] - F[a, d]) > 1e-4 * np.abs(Fm).max()
