"""Pins for the oracle's interpolation from a general (nonnested) coarse mesh
(Sec. 3.2, Algorithm 1): on the uniform Kuhn mesh it equals the closed-form
location already pinned by the nested Galerkin identities; on a jittered
coarse mesh it is a partition of unity and reproduces linear functions
wherever the containing coarse element has no boundary vertex."""
import numpy as np

from ks_inputs import make_workload, freudenthal_mesh, jittered_coarse_mesh
from oracle.coarse import coarse_interpolation, interpolation_in_mesh


def _fine_points():
    w = make_workload("small_molecule", n=6)       # moved P2 mesh of [-15, 15]^3
    return w.mesh.coords[w.mesh.interior], w.mesh.L


def test_general_location_equals_closed_form_on_uniform_coarse_mesh():
    x, L = _fine_points()
    for n_H in (3, 4):
        cm = freudenthal_mesh(n_H, L, 1)
        P_gen = interpolation_in_mesh(x, cm.coords, cm.elems, cm.dirichlet)
        P_cf = coarse_interpolation(x, L, n_H)
        assert P_gen.shape == P_cf.shape
        assert np.abs(P_gen - P_cf).max() < 1e-13


def test_jittered_coarse_mesh_partition_of_unity_and_linears():
    x, L = _fine_points()
    cm = jittered_coarse_mesh(4, L, amp=0.3, seed=7)
    P = interpolation_in_mesh(x, cm.coords, cm.elems, cm.dirichlet)
    inner = np.flatnonzero(cm.dirichlet == 0)
    # rows whose support is four interior coarse vertices: full partition of unity
    full = (P > 0).sum(axis=1) == 4
    assert full.sum() > 20
    assert np.abs(P[full].sum(axis=1) - 1.0).max() < 1e-13
    # linear reproduction on those rows: sum_c P[a, c] x_c = x_a
    xr = P[full] @ cm.coords[inner]
    assert np.abs(xr - x[full]).max() < 1e-12
    # every row is a convex combination (nonnegative weights summing to <= 1)
    assert P.min() >= -1e-14 and P.sum(axis=1).max() <= 1.0 + 1e-13
    # the jitter makes the coarse mesh nonnested: weights differ from the uniform mesh
    assert np.abs(P - coarse_interpolation(x, L, 4)).max() > 1e-2
