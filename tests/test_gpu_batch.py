"""Batched form: many independent systems of uneven size solved in one
persistent launch (captured once in a hipGraph, replayed by every solve),
checked system by system against the single-system block solve and the
oracle's block solve."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from ks_inputs.workloads import batched_systems
from oracle.step import KSProblem, initial_guess, block_solve
from oracle.xc import lda_xc

DEV = "cuda:0"
TIGHT = dict(tol_solve=1e-13, tol_inner=1e-11, tol_poisson=1e-13)


def _rel(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _systems(count, n_cap):
    from paper_2404_19249_amd import KSContext
    ws = batched_systems(count, n_cap=n_cap)
    ctxs, psis, lams = [], [], []
    for i, w in enumerate(ws):
        print(f"[case] batch system {i}: n={w.mesh.n} P{w.mesh.order} k={w.k}", flush=True)
        c = KSContext.from_workload(w, **TIGHT)
        th, Psi = initial_guess(KSProblem.from_workload(w), w.k)
        psi = torch.tensor(Psi, device=DEV)
        c.assemble(psi, w.occ, want_fields=False)
        ctxs.append(c); psis.append(psi); lams.append(th)
    return ws, ctxs, psis, lams


def _oracle_operator(w, Psi):
    """S = K/2 + M[V_eff(rho(Psi))] + mu M from the oracle alone."""
    p = KSProblem.from_workload(w)
    rho = p.density(Psi)
    VH, _ = p.hartree_nodes(rho, p.boundary_data(rho), 1e-14)
    _, vxc = lda_xc(rho, p.xc_mode)
    veff = p.vext_q + p.at_quad(VH) + vxc
    return p, (0.5 * p.K_II + p.potential_matrix(veff) + p.mu * p.M_II).tocsr()


@pytest.mark.parametrize("grid", [0, 12])
def test_batched_solve_matches_single_solves(grid):
    from paper_2404_19249_amd import KSBatch
    ws, ctxs, psis, lams = _systems(12, 9)
    refs = [c.block_solve(p, l)[0].cpu().numpy() for c, p, l in zip(ctxs, psis, lams)]
    b = KSBatch(ctxs, [w.k for w in ws], grid=grid)
    print(f"[case] grid={b.grid} teams={b.team} ng={b.ng}", flush=True)
    assert b.grid == (grid if grid else b.grid) and sum(b.team) == b.grid
    if grid == 0:
        ms = b.autotune(psis, lams, rounds=2)
        print(f"[case] tuned {ms:.3f} ms teams={b.team} ng={b.ng}", flush=True)
        assert ms > 0 and sum(b.team) == b.grid and min(b.team) >= 1
    for rep in range(3):
        outs, st = b.block_solve(psis, lams)
        assert st["status"] == 0 and all(s == 0 for s in st["sys_status"])
        for i, (o, r) in enumerate(zip(outs, refs)):
            assert _rel(o.cpu().numpy(), r) < 1e-10, (rep, i)
            assert st["relres"][i] < 1e-12
        assert 0 < max(st["system_seconds"]) <= st["seconds"] * 1.5 + 1e-3
        # eager work between replays
        ctxs[0].block_solve(psis[0], lams[0])
    b.close()


def test_batched_solve_follows_new_inputs_and_matches_oracle():
    from paper_2404_19249_amd import KSBatch
    ws, ctxs, psis, lams = _systems(5, 7)
    b = KSBatch(ctxs, [w.k for w in ws])
    for rep, shift in enumerate([0.0, -0.05]):
        lam2 = [l + shift for l in lams]
        outs, st = b.block_solve(psis, lam2)
        for i, w in enumerate(ws):
            Psi = psis[i].cpu().numpy()
            p, S = _oracle_operator(w, Psi)
            ref, its, _ = block_solve(p, S, Psi, lam2[i], tol=1e-13)
            assert _rel(outs[i].cpu().numpy(), ref) < 1e-10, (rep, i)
            assert abs(st["iters"][i] - int(max(its))) <= 2
    b.close()


def test_batched_row_and_tile_products_agree():
    """Both product forms of the batched kernel -- row products from the CSR
    arrays and halo tiles staged in LDS, at every row block a system can
    take -- give the single-system solutions; a row block that does not exist
    and a lanes-per-row split that does not fit are refused."""
    from paper_2404_19249_amd import KSBatch, KSError
    ws, ctxs, psis, lams = _systems(6, 9)
    n = len(ws)
    refs = [c.block_solve(p, l)[0].cpu().numpy() for c, p, l in zip(ctxs, psis, lams)]
    b = KSBatch(ctxs, [w.k for w in ws], grid=4 * n)   # few workgroups: room in LDS
    tiled = 0
    for br in (0, 32, 64, 85, 128, 170, 256):
        t = [0] * n
        for i in range(n if br else 0):
            t[i] = br
            try:
                b.set_layout(tile=t)
            except KSError:
                t[i] = 0
        b.set_layout(tile=t)
        assert b.tile == t
        tiled += sum(1 for x in t if x)
        print(f"[case] rows per tile {br}: tiled {t}", flush=True)
        outs, st = b.block_solve(psis, lams)
        assert st["status"] == 0
        for i, (o, r) in enumerate(zip(outs, refs)):
            assert _rel(o.cpu().numpy(), r) < 1e-10, (br, i)
            assert st["relres"][i] < 1e-12
    assert tiled >= n
    with pytest.raises(KSError):
        b.set_layout(tile=[77] * n)
    with pytest.raises(KSError):
        b.set_layout(ng=[3] * n)
    b.close()


def test_batch_rejects_bad_arguments():
    from paper_2404_19249_amd import KSBatch, KSError
    ws, ctxs, psis, lams = _systems(2, 6)
    with pytest.raises(KSError):
        KSBatch(ctxs, [ws[0].k, 99])
    with pytest.raises(KSError):
        KSBatch(ctxs, [w.k for w in ws], grid=1)
