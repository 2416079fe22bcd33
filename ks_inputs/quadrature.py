"""Conical-product (Stroud) quadrature on the reference tetrahedron.

The paper does not state its quadrature; this rule is the input that fixes
where V_eff, rho and the potential matrices are evaluated.  With n points per
direction the rule has n^3 points and integrates polynomials of total degree
<= 2n-1 exactly over the unit tetrahedron {x, y, z >= 0, x + y + z <= 1}:

    x = a,  y = (1-a) b,  z = (1-a)(1-b) c,   dV = (1-a)^2 (1-b) da db dc

with Gauss-Jacobi rules in a (weight (1-a)^2), b (weight (1-b)) and
Gauss-Legendre in c, each computed by the Golub-Welsch eigenvalue method.

Output: barycentric coordinates [n_q][4] = (1-x-y-z, x, y, z) and weights
[n_q] summing to 1/6 (the reference volume).
"""
from dataclasses import dataclass
from math import gamma
import numpy as np


@dataclass
class QuadRule:
    bary: np.ndarray   # [n_q][4]
    w: np.ndarray      # [n_q], sums to 1/6

    @property
    def n_q(self):
        return self.w.shape[0]

    @property
    def points(self):
        return self.bary[:, 1:4]


def gauss_jacobi_01(n: int, alpha: float):
    """n-point Gauss rule on [0,1] for the weight (1-t)^alpha (Golub-Welsch)."""
    a_, b_ = float(alpha), 0.0
    k = np.arange(n, dtype=np.float64)
    s = 2.0 * k + a_ + b_
    diag = np.empty(n)
    with np.errstate(divide="ignore", invalid="ignore"):
        diag[:] = (b_ * b_ - a_ * a_) / (s * (s + 2.0))
    diag[0] = (b_ - a_) / (a_ + b_ + 2.0)
    kk = np.arange(1, n, dtype=np.float64)
    ss = 2.0 * kk + a_ + b_
    off2 = 4.0 * kk * (kk + a_) * (kk + b_) * (kk + a_ + b_) / (ss * ss * (ss + 1.0) * (ss - 1.0))
    T = np.diag(diag) + np.diag(np.sqrt(off2), 1) + np.diag(np.sqrt(off2), -1)
    ev, V = np.linalg.eigh(T)
    mu0 = 2.0 ** (a_ + b_ + 1.0) * gamma(a_ + 1.0) * gamma(b_ + 1.0) / gamma(a_ + b_ + 2.0)
    w = mu0 * V[0, :] ** 2
    # map [-1,1] -> [0,1]: (1-t) = 2(1-x), dt = 2 dx
    x = 0.5 * (ev + 1.0)
    w = w / 2.0 ** (a_ + 1.0)
    return x, w


def conical_rule(n: int) -> QuadRule:
    xa, wa = gauss_jacobi_01(n, 2.0)
    xb, wb = gauss_jacobi_01(n, 1.0)
    xc, wc = gauss_jacobi_01(n, 0.0)
    pts, ws = [], []
    for i in range(n):
        for j in range(n):
            for l in range(n):
                a, b, c = xa[i], xb[j], xc[l]
                x = a
                y = (1.0 - a) * b
                z = (1.0 - a) * (1.0 - b) * c
                pts.append((1.0 - x - y - z, x, y, z))
                ws.append(wa[i] * wb[j] * wc[l])
    return QuadRule(bary=np.array(pts, dtype=np.float64), w=np.array(ws, dtype=np.float64))


def rule_for_order(order: int) -> QuadRule:
    """8 points (degree 3) for P1, 27 points (degree 5) for P2: both make the
    mass matrix exact and put the potential at enough points for the P2
    product phi_a phi_b V."""
    return conical_rule(2 if order == 1 else 3)
