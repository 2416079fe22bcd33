"""ORACLE (test infrastructure only): the Hessian metric of Sec. 3.2 and a
metric-driven node mover standing in for the remesher of Algorithm 2.

Sec. 3.2 moves the mesh by a metric built from the Hessian of the adaptive
function u = sqrt(rho) (Algorithm 2 uses sqrt(rho_h) of the current level):
the eigen-decomposition H = R Lambda R^T at every node, each eigenvalue
replaced by lambda~_i = min(max(C_d |lambda_i| / eps, 1 / h_max^2),
1 / h_min^2) with C_d = 1/2 (d / (d + 1))^2 (eq. m2), and M = R Lambda~ R^T
(eq. m1).  The paper hands M to Mshmet/Mmg3d; those tools are not part of
this work, so the steps below are readings:

* u at the nodes of a P1 mesh: u_a = sqrt(sum_i f_i psi_i(x_a)^2), zero at
  Dirichlet nodes (psi vanishes there).
* Hessian recovery: the gradient of the P1 interpolant is constant per
  element; its lumped-mass L2 projection onto P1 is the volume-weighted
  average G_a = sum_{e ni a} |e| grad u_e / sum_{e ni a} |e|.  Applying the
  same projection to each component of G gives D, and H_a = (D_a + D_a^T)/2.
* Node mover: the metric spring energy E(x) = sum over mesh edges (a, b) of
  (x_b - x_a)^T Mbar_ab (x_b - x_a), Mbar_ab = (M_a + M_b) / 2, the metric
  carried by the nodes.  A sweep moves every free node toward the minimiser
  of E over that node with the others fixed,
      x_a <- (1 - omega) x_a + omega (sum_b Mbar_ab)^{-1} sum_b Mbar_ab x_b,
  all nodes from the previous positions (Jacobi); Dirichlet nodes stay.  A
  sweep that would leave an element with det J <= 0 is redone with omega
  halved (at most 20 times).  Edges that are long in the metric pull
  hardest, so nodes gather where M is large (where u curves).
"""
import numpy as np

C_D3 = 0.5 * (3.0 / 4.0) ** 2  # C_d of the L-infinity interpolation estimate, d = 3


def nodal_sqrt_density(n_nodes, dirichlet, psi_int, occ):
    """u = sqrt(sum_i f_i psi_i^2) at every node; psi_int [N][k] over the
    non-Dirichlet nodes in ascending order."""
    u = np.zeros(n_nodes)
    inner = np.flatnonzero(np.asarray(dirichlet) == 0)
    psi = np.asarray(psi_int, dtype=np.float64)
    u[inner] = np.sqrt((psi ** 2) @ np.asarray(occ, dtype=np.float64))
    return u


def _volumes_and_gradients(coords, tets):
    X = coords[tets]                                             # [n_e][4][3]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)                                      # rows: grad lambda_1..3
    gl = np.empty((tets.shape[0], 4, 3))
    gl[:, 1:] = Jinv
    gl[:, 0] = -Jinv.sum(axis=1)
    return det / 6.0, gl


def recover_gradient(coords, tets, u):
    """Volume-weighted average of the element gradients of the P1
    interpolant of u (one column of values per field: u [n_nodes] or
    [n_nodes][m]); returns [n_nodes][3] or [n_nodes][m][3]."""
    coords = np.asarray(coords, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)[:, :4]
    vol, gl = _volumes_and_gradients(coords, tets)
    U = np.asarray(u, dtype=np.float64)
    single = U.ndim == 1
    if single:
        U = U[:, None]
    ge = np.einsum("eam,eax->emx", U[tets], gl)                  # [n_e][m][3]
    num = np.zeros((coords.shape[0], U.shape[1], 3))
    den = np.zeros(coords.shape[0])
    for a in range(4):
        np.add.at(num, tets[:, a], vol[:, None, None] * ge)
        np.add.at(den, tets[:, a], vol)
    G = num / den[:, None, None]
    return G[:, 0, :] if single else G


def recover_hessian(coords, tets, u):
    """Symmetrised recovered gradient of the recovered gradient: [n_nodes][3][3]."""
    G = recover_gradient(coords, tets, u)                        # [n][3]
    D = recover_gradient(coords, tets, G)                        # [n][3 (component)][3 (derivative)]
    return 0.5 * (D + np.transpose(D, (0, 2, 1)))


def metric_from_hessian(H, eps, h_min, h_max):
    """Eqs. m1-m2: M = R Lambda~ R^T per node."""
    lam, R = np.linalg.eigh(np.asarray(H, dtype=np.float64))
    lt = np.minimum(np.maximum(C_D3 * np.abs(lam) / eps, 1.0 / h_max ** 2), 1.0 / h_min ** 2)
    return np.einsum("nij,nj,nkj->nik", R, lt, R)


def mesh_edges(tets):
    """Unique edges (a < b) of a tetrahedral mesh."""
    t = np.asarray(tets, dtype=np.int64)[:, :4]
    e = np.concatenate([t[:, [i, j]] for i in range(4) for j in range(i + 1, 4)], axis=0)
    e.sort(axis=1)
    return np.unique(e, axis=0)


def spring_energy(coords, edges, M):
    d = coords[edges[:, 1]] - coords[edges[:, 0]]
    Mb = 0.5 * (M[edges[:, 0]] + M[edges[:, 1]])
    return float(np.einsum("ei,eij,ej->", d, Mb, d))


def min_det(coords, tets):
    t = np.asarray(tets, dtype=np.int64)[:, :4]
    X = coords[t]
    J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
    return float(np.linalg.det(J).min())


def move_nodes(coords, tets, M, fixed, omega=0.5, sweeps=1, max_halvings=20):
    """Damped Jacobi sweeps of the metric spring mover.  Returns the new
    coordinates and the number of halvings of omega over all sweeps."""
    x = np.array(coords, dtype=np.float64)
    edges = mesh_edges(tets)
    free = np.asarray(fixed) == 0
    halvings = 0
    for _ in range(sweeps):
        Mb = 0.5 * (M[edges[:, 0]] + M[edges[:, 1]])             # [n_edges][3][3]
        A = np.zeros((x.shape[0], 3, 3))
        b = np.zeros((x.shape[0], 3))
        for s, t in ((0, 1), (1, 0)):
            np.add.at(A, edges[:, s], Mb)
            np.add.at(b, edges[:, s], np.einsum("eij,ej->ei", Mb, x[edges[:, t]]))
        target = x.copy()
        target[free] = np.linalg.solve(A[free], b[free][:, :, None])[:, :, 0]
        w = omega
        for _h in range(max_halvings + 1):
            xn = x.copy()
            xn[free] = (1.0 - w) * x[free] + w * target[free]
            if min_det(xn, tets) > 0.0:
                break
            w *= 0.5
            halvings += 1
        else:
            raise RuntimeError("no valid step: every damped move inverts an element")
        x = xn
    return x, halvings
