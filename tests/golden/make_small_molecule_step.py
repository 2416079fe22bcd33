"""Write tests/golden/small_molecule_32_step0.json: one step of Algorithm 3
computed by the CPU oracle on the full-size small-molecule workload (P2 on
32^3 hexes, N = 250,047, k = 5) from the coarse Ritz initial guess, with the
sub-problems solved tightly.  Stored: the initial-guess eigenvalues, the
step's eigenvalues and energies, its iteration counts, and F_B, F_A (the
pencil of eq. st1 in the last inner iteration) as diagonals plus seeded
sampled entries.  Imports only the oracle and the seeded input generators.

Usage: python tests/golden/make_small_molecule_step.py   (about 10 minutes)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from ks_inputs import make_workload                              # noqa: E402
from oracle.step import KSProblem, initial_guess, ks_scf_step    # noqa: E402

TOL = dict(tol_solve=1e-12, tol_inner=1e-11, tol_poisson=1e-13)
N_SAMPLES = 96


def main():
    t0 = time.time()
    w = make_workload("small_molecule")
    p = KSProblem.from_workload(w)
    th0, Psi0 = initial_guess(p, w.k)
    r = ks_scf_step(p, Psi0, th0, max_inner=100, want_eks=False, **TOL)
    m = r.FB.shape[0]
    rng = np.random.default_rng(20240429)
    ij = rng.integers(0, m, size=(N_SAMPLES, 2))
    out = {
        "workload": "small_molecule (P2, 32^3 hexes, seed 2), step 0 from the coarse Ritz guess",
        "tolerances": TOL,
        "N": int(p.N), "k": int(w.k), "m": int(m), "mu": float(p.mu),
        "lambda0": [float(x) for x in th0],
        "lambda": [float(x) for x in r.lam],
        "theta_next": [float(x) for x in r.theta_all[w.k:w.k + 5]],
        "energies": {k: float(v) for k, v in r.energies.items()},
        "inner_iters": int(r.inner_iters),
        "res_inner": float(r.extra["res_inner"]),
        "rank": int(r.rank),
        "solve_iters": [int(x) for x in r.solve_iters],
        "FB_diag": [float(x) for x in np.diag(r.FB)],
        "FA_diag": [float(x) for x in np.diag(r.FA)],
        "sample_ij": ij.tolist(),
        "FB_samples": [float(r.FB[i, j]) for i, j in ij],
        "FA_samples": [float(r.FA[i, j]) for i, j in ij],
        "FB_fro": float(np.linalg.norm(r.FB)),
        "FA_fro": float(np.linalg.norm(r.FA)),
        "oracle_seconds": time.time() - t0,
    }
    path = os.path.join(HERE, "small_molecule_32_step0.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, out["lambda"], out["inner_iters"], f"{out['oracle_seconds']:.0f}s")


if __name__ == "__main__":
    main()
