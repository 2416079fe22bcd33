"""Pins for the oracle's quadrature, element matrices and global assembly.

Each check compares against something other than the oracle's own formula:
exact integrals of monomials over the reference tetrahedron, the classical
closed-form P1 element matrices, the barycentric-monomial integration formula
for P2, and exact identities of the assembled matrices."""
from itertools import product
from math import factorial

import numpy as np
import pytest

from ks_inputs import conical_rule, freudenthal_mesh, move_nodes_toward_nuclei, make_workload
from ks_inputs.quadrature import rule_for_order
from oracle import fe


# ---------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n", [2, 3])
def test_quadrature_exact_on_monomials(n):
    q = conical_rule(n)
    x, y, z = q.points.T
    for a, b, c in product(range(2 * n), repeat=3):
        if a + b + c > 2 * n - 1:
            continue
        exact = factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)
        assert abs(np.sum(q.w * x ** a * y ** b * z ** c) - exact) < 1e-15
    assert abs(q.w.sum() - 1.0 / 6.0) < 1e-15
    assert np.all(q.w > 0) and np.all(q.bary > 0)


def test_quadrature_not_exact_beyond_degree():
    q = conical_rule(2)
    x = q.points[:, 0]
    exact = factorial(4) / factorial(7)
    assert abs(np.sum(q.w * x ** 4) - exact) > 1e-6


# ------------------------------------------------------------ element level
def _random_tets(n, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 4, 3))
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], 2)
    s = np.linalg.det(J) < 0
    X[s, 2], X[s, 3] = X[s, 3].copy(), X[s, 2].copy()
    return X


def _bary_monomial_integral(expo, vol):
    """int_T prod lambda_i^{a_i} = 3! |T| prod a_i! / (sum a_i + 3)!"""
    num = np.prod([factorial(a) for a in expo])
    return 6.0 * vol * num / factorial(sum(expo) + 3)


def _p2_poly(a):
    """P2 basis function a as {exponent tuple: coeff} in barycentric monomials."""
    if a < 4:
        e2 = [0, 0, 0, 0]; e2[a] = 2
        e1 = [0, 0, 0, 0]; e1[a] = 1
        return {tuple(e2): 2.0, tuple(e1): -1.0}
    i, j = fe.P2_EDGES[a - 4]
    e = [0, 0, 0, 0]; e[i] = 1; e[j] = 1
    return {tuple(e): 4.0}


def _poly_mul(p, q):
    out = {}
    for ea, ca in p.items():
        for eb, cb in q.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0.0) + ca * cb
    return out


def _poly_diff(p, v):
    out = {}
    for e, c in p.items():
        if e[v] > 0:
            ee = list(e); ee[v] -= 1
            out[tuple(ee)] = out.get(tuple(ee), 0.0) + c * e[v]
    return out


def _integrate(p, vol):
    return sum(c * _bary_monomial_integral(e, vol) for e, c in p.items())


def test_p1_element_matrices_closed_form():
    X = _random_tets(20)
    elems = np.arange(80).reshape(20, 4)
    coords = X.reshape(-1, 3)
    J, det, gl = fe.element_geometry(coords, elems)
    q = rule_for_order(1)
    M = fe.element_matrices(1, q, det, gl, kind="mass")
    K = fe.element_matrices(1, q, det, gl, kind="stiffness")
    vol = det / 6.0
    Mref = vol[:, None, None] * (np.ones((4, 4)) + np.eye(4))[None] / 20.0
    Kref = vol[:, None, None] * np.einsum("eid,ejd->eij", gl, gl)
    assert np.allclose(M, Mref, rtol=1e-13, atol=0)
    assert np.allclose(K, Kref, rtol=1e-12, atol=1e-14 * np.abs(Kref).max())
    # independent gradients: grad lambda solves lambda_i(X_j) = delta_ij
    for e in range(3):
        A = np.hstack([X[e], np.ones((4, 1))])
        coef = np.linalg.solve(A, np.eye(4))       # columns: (grad, const) of lambda_i
        assert np.allclose(coef[:3].T, gl[e], atol=1e-12)


def test_p2_element_matrices_by_monomial_formula():
    X = _random_tets(6, seed=1)
    elems = np.arange(24).reshape(6, 4)
    coords = X.reshape(-1, 3)
    J, det, gl = fe.element_geometry(coords, elems)
    q = rule_for_order(2)
    M = fe.element_matrices(2, q, det, gl, kind="mass")
    K = fe.element_matrices(2, q, det, gl, kind="stiffness")
    for e in range(6):
        vol = det[e] / 6.0
        G = gl[e] @ gl[e].T                           # grad lambda_v . grad lambda_w
        for a in range(10):
            for b in range(10):
                pa, pb = _p2_poly(a), _p2_poly(b)
                m = _integrate(_poly_mul(pa, pb), vol)
                k = 0.0
                for v in range(4):
                    for w in range(4):
                        k += G[v, w] * _integrate(_poly_mul(_poly_diff(pa, v), _poly_diff(pb, w)), vol)
                assert abs(M[e, a, b] - m) < 1e-13 * max(1.0, abs(m))
                assert abs(K[e, a, b] - k) < 1e-11 * max(1.0, np.abs(K[e]).max())


def test_potential_matrix_of_constant_is_mass():
    w = make_workload("small_molecule", n=3)
    m = w.mesh
    J, det, gl = fe.element_geometry(m.coords, m.elems)
    Me = fe.element_matrices(2, w.quad, det, gl, kind="mass")
    V = np.full((m.n_elems, w.quad.n_q), 2.5)
    MVe = fe.element_matrices(2, w.quad, det, gl, V=V, kind="potential")
    assert np.allclose(MVe, 2.5 * Me, rtol=1e-14, atol=0)


# ----------------------------------------------------------------- global
@pytest.mark.parametrize("order,moved", [(1, False), (1, True), (2, False), (2, True)])
def test_global_invariants(order, moved):
    L = 3.0
    mesh = freudenthal_mesh(4, L, order)
    if moved:
        mesh = move_nodes_toward_nuclei(mesh, [[0.4, -0.3, 0.2]], a=0.5, s=1.0)
    q = rule_for_order(order)
    J, det, gl = fe.element_geometry(mesh.coords, mesh.elems)
    K = fe.assemble(mesh.n_nodes, mesh.elems, fe.element_matrices(order, q, det, gl, kind="stiffness"))
    M = fe.assemble(mesh.n_nodes, mesh.elems, fe.element_matrices(order, q, det, gl, kind="mass"))
    Kd, Md = K.toarray(), M.toarray()
    assert np.allclose(Kd, Kd.T, atol=1e-13)
    assert np.allclose(Md, Md.T, atol=1e-15)
    one = np.ones(mesh.n_nodes)
    assert np.abs(K @ one).max() < 1e-12
    assert abs(one @ (M @ one) - (2 * L) ** 3) < 1e-11
    x = mesh.coords[:, 0]
    y = mesh.coords[:, 1]
    # u = x is in the space: int |grad x|^2 = |Omega|
    assert abs(x @ (K @ x) - (2 * L) ** 3) < 1e-10
    # int x y = 0 on the symmetric cube; int x^2 = (2L)^2 * 2L^3/3
    assert abs(x @ (M @ y)) < 1e-11
    assert abs(x @ (M @ x) - (2 * L) ** 2 * 2 * L ** 3 / 3) < 1e-10
    if order == 2:
        u = x * x   # quadratics are in the P2 space on affine elements
        assert abs(u @ (K @ u) - 4 * (2 * L) ** 2 * 2 * L ** 3 / 3) < 1e-9
        assert abs(u @ (M @ one) - (2 * L) ** 2 * 2 * L ** 3 / 3) < 1e-10
    I = mesh.interior
    KII = Kd[np.ix_(I, I)]
    assert np.linalg.eigvalsh(KII).min() > 0
    assert np.linalg.eigvalsh(Md).min() > 0


def test_inverted_element_rejected():
    mesh = freudenthal_mesh(2, 1.0, 1)
    el = mesh.elems.copy()
    el[3, [2, 3]] = el[3, [3, 2]]
    with pytest.raises(ValueError):
        fe.element_geometry(mesh.coords, el)


def test_mesh_sizes_match_lattice_counts():
    """Interior DOFs and nonzeros of the Freudenthal lattice (P1: 15 per
    interior row; P2 mixes 65/27/19/27 per vertex/axis/face/body node)."""
    from oracle.step import KSProblem
    p = KSProblem.from_workload(make_workload("hydrogen"))
    assert p.N == 3375 and p.K_II.nnz == 45403
    w = make_workload("small_molecule", n=4)
    p2 = KSProblem.from_workload(w)
    assert p2.N == 7 ** 3
    m = freudenthal_mesh(32, 15.0, 2)
    assert m.n_nodes == 274625 and len(m.interior) == 250047 and m.n_elems == 196608
