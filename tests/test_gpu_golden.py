"""The small-molecule workload at full size (P2, 32^3 hexes, N = 250,047,
k = 5): one step of Algorithm 3 from the coarse Ritz guess against the
oracle's step stored in tests/golden/small_molecule_32_step0.json (written by
tests/golden/make_small_molecule_step.py, which imports only the oracle and
the seeded inputs).  Both sides solve their sub-problems tightly, so the
comparison is at the FP64 parity tolerance."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

from ks_inputs import make_workload

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "small_molecule_32_step0.json")


def _rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_small_molecule_full_size_step_matches_golden():
    from paper_2404_19249_amd import KSContext
    g = json.load(open(GOLDEN))
    w = make_workload("small_molecule")
    print("[case] small_molecule full size, golden step 0", flush=True)
    t = g["tolerances"]
    ctx = KSContext.from_workload(w, tol_solve=t["tol_solve"], tol_inner=t["tol_inner"],
                                  tol_poisson=t["tol_poisson"], max_it_inner=100)
    assert ctx.N == g["N"] and abs(ctx.mu - g["mu"]) < 1e-12 * g["mu"]
    psi, lam0 = ctx.initial_guess(w.k)
    assert _rel(lam0, g["lambda0"]) < 1e-11
    lam, rep = ctx.scf_step(psi, lam0, w.occ, precision="fp64")
    print({"lambda": list(lam), "golden": g["lambda"], "inner": rep["inner_iters"],
           "golden_inner": g["inner_iters"]}, flush=True)
    assert rep["status"] == 0 and rep["res_inner"] < t["tol_inner"]
    assert rep["rank"] == g["rank"]
    assert _rel(lam, g["lambda"]) < 1e-10
    assert abs(rep["E_total"] - g["energies"]["total"]) < 1e-10 * abs(g["energies"]["total"])
    for key, name in (("FB", "FB"), ("FA", "FA")):
        m = g["m"]
        F = ctx.debug_buffer(name, m * m).cpu().numpy().reshape(m, m)
        scale = np.abs(np.asarray(g[f"{key}_diag"])).max()
        assert np.abs(np.diag(F) - g[f"{key}_diag"]).max() < 1e-10 * scale, key
        ij = np.asarray(g["sample_ij"])
        assert np.abs(F[ij[:, 0], ij[:, 1]] - g[f"{key}_samples"]).max() < 1e-10 * scale, key
        assert abs(np.linalg.norm(F) - g[f"{key}_fro"]) < 1e-10 * g[f"{key}_fro"], key
    ctx.close()
