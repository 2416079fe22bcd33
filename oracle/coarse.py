"""ORACLE (test infrastructure only): interpolation from the coarse space S_H.

Sec. 3.2 (Algorithm 1) interpolates a coarse P1 function at every fine node
by locating the node in a coarse tetrahedron and evaluating the linear
interpolant with its barycentric coordinates.  The coarse mesh here is the
uniform Kuhn mesh of the same box with n_H hexahedra per side, so point
location is closed-form: the hexahedron by floor(), the Kuhn tetrahedron by
the descending order of the local coordinates (ties broken x before y before
z; by continuity the interpolated value does not depend on the tie-break).

The interpolation matrix P[a][c] = phi^H_c(x_a) over interior fine nodes a
and interior coarse vertices c (S_H is a subspace of H^1_0, so coarse
boundary vertices carry no basis function).
"""
import numpy as np


def coarse_interpolation(x_fine, L, n_H):
    """Dense P [n_fine][(n_H-1)^3] for fine points x_fine [n_fine][3]."""
    h = 2.0 * L / n_H
    t = (np.asarray(x_fine, dtype=np.float64) + L) / h
    cell = np.clip(np.floor(t), 0, n_H - 1).astype(np.int64)
    xi = t - cell
    nf = x_fine.shape[0]
    ni = n_H - 1
    P = np.zeros((nf, ni ** 3))
    for a in range(nf):
        order = sorted(range(3), key=lambda d: (-xi[a, d], d))
        s = xi[a, order]
        lam = [1.0 - s[0], s[0] - s[1], s[1] - s[2], s[2]]
        v = cell[a].copy()
        verts = [v.copy()]
        for d in order:
            v[d] += 1
            verts.append(v.copy())
        for lv, vv in zip(lam, verts):
            if np.any(vv <= 0) or np.any(vv >= n_H):
                continue            # coarse boundary vertex: no basis function
            cid = (vv[0] - 1) + ni * ((vv[1] - 1) + ni * (vv[2] - 1))
            P[a, cid] += lv
    return P


def interpolation_in_mesh(x_fine, coarse_coords, coarse_tets, coarse_dirichlet):
    """Dense P [n_fine][n_inner] for a general coarse P1 tetrahedral mesh, by
    the definition: for every fine point, the coarse element that contains it
    (brute force over all elements: the one whose smallest barycentric
    coordinate is largest), and its barycentric coordinates as the values of
    that element's vertex basis functions.  Coarse vertices with a Dirichlet
    flag carry no basis function; the others are numbered by ascending id."""
    cv = np.asarray(coarse_coords, dtype=np.float64)
    T = np.asarray(coarse_tets, dtype=np.int64)
    inner = np.flatnonzero(np.asarray(coarse_dirichlet) == 0)
    cid = -np.ones(cv.shape[0], dtype=np.int64)
    cid[inner] = np.arange(inner.size)
    X0 = cv[T[:, 0]]
    J = np.stack([cv[T[:, 1]] - X0, cv[T[:, 2]] - X0, cv[T[:, 3]] - X0], axis=2)  # [n_t][3][3]
    Jinv = np.linalg.inv(J)
    x = np.asarray(x_fine, dtype=np.float64)
    P = np.zeros((x.shape[0], inner.size))
    for a in range(x.shape[0]):
        l123 = np.einsum("tij,tj->ti", Jinv, x[a][None, :] - X0)
        lam = np.concatenate([1.0 - l123.sum(axis=1, keepdims=True), l123], axis=1)
        t = int(np.argmax(lam.min(axis=1)))
        for j in range(4):
            c = cid[T[t, j]]
            if c >= 0:
                P[a, c] += lam[t, j]
    return P
