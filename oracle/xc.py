"""ORACLE (test infrastructure only): local density approximation of Sec. 3.1.

Exchange (Kohn-Sham / Dirac form):
    eps_x = -(3/4) (3/pi)^{1/3} rho^{1/3},   V_x = -(3 rho / pi)^{1/3}
Correlation (Perdew-Zunger), r_s = (3 / (4 pi rho))^{1/3}:
    r_s < 1:  eps_c = A ln r_s + B + C r_s ln r_s + D r_s
              V_c   = A ln r_s + (B - A/3) + (2/3) C r_s ln r_s + (1/3)(2D - C) r_s
    r_s >= 1: eps_c = gamma / (1 + beta1 sqrt(r_s) + beta2 r_s)
              V_c   = eps_c (1 + (7/6) beta1 sqrt(r_s) + (4/3) beta2 r_s)
                            / (1 + beta1 sqrt(r_s) + beta2 r_s)
with the constants printed in the paper.  Reading: rho <= 1e-30 gives zero
for every XC quantity (the paper does not treat rho -> 0); r_s = 1 takes the
second branch, as printed.
"""
import numpy as np

A_PZ, B_PZ, C_PZ, D_PZ = 0.0311, -0.048, 0.0020, -0.0116
G_PZ, B1_PZ, B2_PZ = -0.1423, 1.0529, 0.3334
RHO_FLOOR = 1e-30


def lda_xc(rho, mode="x_pz81"):
    """Return (eps_xc, v_xc) at every point; mode in {'none', 'x_only', 'x_pz81'}."""
    rho = np.asarray(rho, dtype=np.float64)
    eps = np.zeros_like(rho)
    v = np.zeros_like(rho)
    if mode == "none":
        return eps, v
    m = rho > RHO_FLOOR
    r = rho[m]
    ex = -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * np.cbrt(r)
    vx = -np.cbrt(3.0 * r / np.pi)
    if mode == "x_only":
        eps[m], v[m] = ex, vx
        return eps, v
    rs = np.cbrt(3.0 / (4.0 * np.pi * r))
    ec = np.empty_like(r)
    vc = np.empty_like(r)
    lo = rs < 1.0
    x = rs[lo]
    lx = np.log(x)
    ec[lo] = A_PZ * lx + B_PZ + C_PZ * x * lx + D_PZ * x
    vc[lo] = A_PZ * lx + (B_PZ - A_PZ / 3.0) + (2.0 / 3.0) * C_PZ * x * lx \
        + (2.0 * D_PZ - C_PZ) * x / 3.0
    hi = ~lo
    x = rs[hi]
    sq = np.sqrt(x)
    den = 1.0 + B1_PZ * sq + B2_PZ * x
    ec[hi] = G_PZ / den
    vc[hi] = ec[hi] * (1.0 + (7.0 / 6.0) * B1_PZ * sq + (4.0 / 3.0) * B2_PZ * x) / den
    eps[m] = ex + ec
    v[m] = vx + vc
    return eps, v
