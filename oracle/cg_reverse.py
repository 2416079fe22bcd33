"""ORACLE (test infrastructure only): reverse mode through the truncated
Jacobi-preconditioned CG of the block BVP solve (eq. Aux_Linear_Problem).

The paper has no derivatives.  The step's implicit adjoint (one adjoint
solve with S) is the derivative of the exact solution S^{-1} B; the solver
stops each column at ||b - S x|| <= tol ||b|| (or an iteration limit), and
the output it returns is that truncated iterate.  This module
differentiates the truncated map itself: every column runs

    r_0 = b - S x_0, z_0 = D^-1 r_0, p_0 = z_0, rho_0 = r_0.z_0
    q_j = S p_j, sigma_j = p_j.q_j, alpha_j = rho_j / sigma_j
    x_{j+1} = x_j + alpha_j p_j, r_{j+1} = r_j - alpha_j q_j
    z_{j+1} = D^-1 r_{j+1}, rho_{j+1} = r_{j+1}.z_{j+1}, beta_j = rho_{j+1} / rho_j
    p_{j+1} = z_{j+1} + beta_j p_j

for its own number of iterations K_c (D = diag S), and for L = sum Xbar * X_K
the reverse sweep returns dL/dS (on the sparsity pattern, the Jacobi
preconditioner's dependence on diag S included) and dL/dB.  With
S = 1/2 K + M[V] + mu M, dS_ab/dV_q = w_q |J| phi_a(x_q) phi_b(x_q) on the
element of q, so dL/dV_q = w_q |J| sum_ab Sbar_ab phi_a(x_q) phi_b(x_q).
Written from the recurrence above by the chain rule, step by step in
reverse order (no stored adjoint of x: xbar stays Xbar through the sweep).
"""
import numpy as np


def truncated_pcg(S, B, X0, tol, max_it):
    """Per-column Jacobi-PCG with the solver's stopping rule; returns X,
    the per-column iteration counts and the per-column scalar histories."""
    S = S.tocsr()
    d = S.diagonal()
    N, k = B.shape
    X = np.array(X0, dtype=np.float64, copy=True)
    R = B - S @ X
    Z = R / d[:, None]
    P = Z.copy()
    rho = np.einsum("ij,ij->j", R, Z)
    bn = np.linalg.norm(B, axis=0)
    active = np.linalg.norm(R, axis=0) > tol * bn
    hist = []
    for _ in range(max_it):
        if not active.any():
            break
        Q = S @ P
        sig = np.einsum("ij,ij->j", P, Q)
        alpha = np.where(active, rho / np.where(active, sig, 1.0), 0.0)
        X = X + alpha * P
        R = R - alpha * Q
        Zn = R / d[:, None]
        rho_n = np.einsum("ij,ij->j", R, Zn)
        beta = np.where(active, rho_n / rho, 0.0)
        hist.append({"active": active.copy(), "alpha": alpha, "beta": beta, "rho": rho.copy(), "sigma": sig})
        P = np.where(active, Zn + beta * P, P)
        rho = np.where(active, rho_n, rho)
        active = active & (np.linalg.norm(R, axis=0) > tol * bn)
    iters = np.array([sum(h["active"][c] for h in hist) for c in range(k)])
    return X, iters, hist


def truncated_pcg_vjp(S, B, X0, tol, max_it, Xbar):
    """dL/dS as a dense matrix (all entries; only the pattern of S is used
    by a caller) and dL/dB for L = sum(Xbar * X_K)."""
    S = S.tocsr()
    d = S.diagonal()
    N, k = B.shape
    X0 = np.asarray(X0, dtype=np.float64)
    # forward, keeping every iterate (small problems)
    R = B - S @ X0
    Z = R / d[:, None]
    P = Z.copy()
    rho = np.einsum("ij,ij->j", R, Z)
    bn = np.linalg.norm(B, axis=0)
    active = np.linalg.norm(R, axis=0) > tol * bn
    Rs, Ps, steps = [R.copy()], [P.copy()], []
    for _ in range(max_it):
        if not active.any():
            break
        Q = S @ P
        sig = np.einsum("ij,ij->j", P, Q)
        alpha = np.where(active, rho / np.where(active, sig, 1.0), 0.0)
        R = R - alpha * Q
        Zn = R / d[:, None]
        rho_n = np.einsum("ij,ij->j", R, Zn)
        beta = np.where(active, rho_n / rho, 0.0)
        steps.append((active.copy(), alpha, beta, rho.copy(), sig))
        P = np.where(active, Zn + beta * P, P)
        rho = np.where(active, rho_n, rho)
        Rs.append(R.copy())
        Ps.append(P.copy())
        active = active & (np.linalg.norm(R, axis=0) > tol * bn)
    # reverse sweep
    xbar = np.asarray(Xbar, dtype=np.float64)
    Sbar = np.zeros((N, N))
    dbar = np.zeros(N)
    rbar = np.zeros((N, k))
    pbar = np.zeros((N, k))
    rhobar = np.zeros(k)
    for j in range(len(steps) - 1, -1, -1):
        act, alpha, beta, rho_j, sig = steps[j]
        a = act.astype(float)
        p, r1 = Ps[j], Rs[j + 1]
        q = S @ p
        z1 = r1 / d[:, None]
        # p_{j+1} = z_{j+1} + beta p_j
        zbar = a * pbar
        betabar = a * np.einsum("ij,ij->j", pbar, p)
        pbar = np.where(act, beta * pbar, pbar)
        # beta = rho_{j+1} / rho_j ; rhobar currently holds d/d rho_{j+1}
        rho1bar = a * (rhobar + betabar / np.where(act, rho_j, 1.0))
        rhojbar = -a * betabar * beta / np.where(act, rho_j, 1.0)
        # rho_{j+1} = r_{j+1}.z_{j+1}
        rbar = rbar + rho1bar * z1
        zbar = zbar + rho1bar * r1
        # z_{j+1} = D^-1 r_{j+1}
        rbar = rbar + zbar / d[:, None]
        dbar -= np.sum(zbar * z1, axis=1) / d
        # r_{j+1} = r_j - alpha q ; x_{j+1} = x_j + alpha p
        alphabar = a * (-np.einsum("ij,ij->j", rbar, q) + np.einsum("ij,ij->j", xbar, p))
        qbar = -alpha * rbar
        pbar = pbar + alpha * xbar
        # alpha = rho_j / sigma_j ; sigma = p.q
        rhojbar = rhojbar + a * alphabar / np.where(act, sig, 1.0)
        sigbar = -a * alphabar * alpha / np.where(act, sig, 1.0)
        pbar = pbar + sigbar * q
        qbar = qbar + sigbar * p
        # q = S p
        pbar = pbar + S @ qbar
        Sbar += qbar @ p.T
        rhobar = np.where(act, rhojbar, rhobar)
    # start: rho_0 = r_0.z_0, p_0 = z_0, z_0 = D^-1 r_0, r_0 = b - S x_0
    r0 = Rs[0]
    z0 = r0 / d[:, None]
    rbar = rbar + rhobar * z0
    zbar = rhobar * r0 + pbar
    rbar = rbar + zbar / d[:, None]
    dbar -= np.sum(zbar * z0, axis=1) / d
    Sbar -= rbar @ X0.T
    Sbar[np.arange(N), np.arange(N)] += dbar
    return Sbar, rbar


def potential_gradient(prob, Sbar):
    """dL/dV_q = dV_q sum_ab Sbar_ab phi_a(x_q) phi_b(x_q) over the interior
    local nodes of the element of q (S = ... + M[V] on the interior rows and
    columns, M[V]_ab = sum_q dV_q V_q phi_a phi_b)."""
    from .fe import basis_tables
    phi, _ = basis_tables(prob.order, prob.quad.bary)            # [n_q][n_loc]
    n2i = -np.ones(prob.n_nodes, dtype=np.int64)
    n2i[prob.interior] = np.arange(prob.interior.size)
    idx = n2i[prob.elems]                                        # [n_e][n_loc], -1 on the boundary
    ok = idx >= 0
    safe = np.where(ok, idx, 0)
    blk = Sbar[safe[:, :, None], safe[:, None, :]] * (ok[:, :, None] & ok[:, None, :])
    return np.einsum("qa,eab,qb->eq", phi, blk, phi) * prob.dV
