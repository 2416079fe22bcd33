"""The bench workload at full size (P2, 64^3 hexes, N = 2,048,383, k = 24) in
the launch configuration bench.py times.

The oracle cannot assemble or solve the whole problem in test time, so:
* sampled rows of K, M and A^L = K/2 + M[V_ext] are recomputed one by one from
  the oracle's element routines over the elements that touch each sampled
  node;
* the block solves are checked by an independent FP64 recomputation of
  ||b - S x|| / ||b|| on the host (scipy, from the exported CSR);
* one SCF step is checked through properties that hold at any size:
  M-orthonormality of the new orbitals and conservation of the charge."""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

from ks_inputs import make_workload
from oracle.fe import element_geometry, element_matrices, quad_points, quad_weights
from oracle.step import external_potential

DEV = "cuda:0"


@pytest.fixture(scope="module")
def full():
    from paper_2404_19249_amd import KSContext
    print("[case] mixed full size", flush=True)
    w = make_workload("mixed")
    ctx = KSContext.from_workload(w, tol_solve=1e-8, tol_inner=1e-8, tol_poisson=1e-10)
    interior = np.flatnonzero(w.mesh.dirichlet == 0)
    yield w, ctx, interior
    ctx.close()


def _csr(ctx, which):
    rp, cl, vl = ctx.export_operator(which)
    return sp.csr_matrix((vl, cl, rp), shape=(ctx.N, ctx.N))


def _sampled_rows(w, interior, rows, kind):
    """Rows `rows` (interior indices) of the operator `kind` over interior
    columns, summed from the oracle's element matrices of the elements that
    touch those nodes."""
    m = w.mesh
    nat = -np.ones(m.coords.shape[0], dtype=np.int64)
    nat[interior] = np.arange(interior.size)
    nodes = interior[rows]
    sel = np.flatnonzero(np.isin(m.elems, nodes).any(axis=1))
    el = m.elems[sel]
    _, det, gl = element_geometry(m.coords, el)
    if kind == "AL":
        V = external_potential(quad_points(m.coords, el, w.quad.bary), w.atoms.Z, w.atoms.R)
        Ae = 0.5 * element_matrices(m.order, w.quad, det, gl, kind="stiffness") + \
            element_matrices(m.order, w.quad, det, gl, V=V, kind="potential")
    else:
        Ae = element_matrices(m.order, w.quad, det, gl, kind=kind)
    want = {int(r): {} for r in rows}
    rowset = set(int(r) for r in rows)
    for e in range(el.shape[0]):
        for a in range(el.shape[1]):
            ra = int(nat[el[e, a]])
            if ra not in rowset:
                continue
            for b in range(el.shape[1]):
                cb = int(nat[el[e, b]])
                if cb >= 0:
                    want[ra][cb] = want[ra].get(cb, 0.0) + Ae[e, a, b]
    return want


@pytest.mark.parametrize("which,kind", [(1, "stiffness"), (2, "mass"), (3, "AL")])
def test_sampled_operator_rows_match_oracle(full, which, kind):
    w, ctx, interior = full
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(ctx.N, 48, replace=False))
    rows = np.concatenate([rows, [0, ctx.N - 1]])  # the first and last rows (ragged block tail)
    A = _csr(ctx, which)
    want = _sampled_rows(w, interior, rows, kind)
    scale = np.abs(A.data).max()
    for r in rows:
        got = A.getrow(int(r))
        ref = want[int(r)]
        assert sorted(got.indices.tolist()) == sorted(ref.keys()), (which, r)
        for c, v in zip(got.indices, got.data):
            assert abs(v - ref[int(c)]) < 1e-12 * scale, (which, r, c)


def test_block_solves_reach_tolerance_recomputed_on_host(full):
    w, ctx, interior = full
    psi, lam = ctx.initial_guess(w.k)
    ctx.assemble(psi, w.occ, want_fields=False)
    S = _csr(ctx, 0)
    M = _csr(ctx, 2)
    P = psi.cpu().numpy()
    B = (M @ P) * (lam + ctx.mu)[None, :]
    bn = np.linalg.norm(B, axis=0)
    sols = {}
    for prec in ("fp64", "mixed"):
        X, st = ctx.block_solve(psi, lam, prec)
        X = X.cpu().numpy()
        rel = np.linalg.norm(B - S @ X, axis=0) / bn
        print(prec, st["iters"][:4], rel.max(), flush=True)
        assert st["converged"]
        assert rel.max() <= 1e-8 * 1.0001, prec
        sols[prec] = X
    d = np.abs(sols["mixed"] - sols["fp64"]).max() / np.abs(sols["fp64"]).max()
    assert d < 1e-6


def test_step_keeps_orthonormality_and_charge(full):
    w, ctx, interior = full
    psi, lam = ctx.initial_guess(w.k)
    rho = torch.empty(ctx.n_elems, ctx.n_q, dtype=torch.float64, device=DEV)
    # the first step from the coarse guess leaves its inner iteration at the
    # iteration cap (as in the benchmark's warm-up); the second converges
    lam, rep = ctx.scf_step(psi, lam, w.occ, rho_out=rho)
    lam, rep = ctx.scf_step(psi, lam, w.occ, rho_out=rho)
    assert rep["res_inner"] < 1e-8
    assert np.all(np.diff(lam) >= -1e-12)
    M = _csr(ctx, 2)
    P = psi.cpu().numpy()
    G = P.T @ (M @ P)
    assert np.abs(G - np.eye(w.k)).max() < 1e-10
    m = w.mesh
    _, det, _ = element_geometry(m.coords, m.elems)
    charge = float(np.sum(quad_weights(det, w.quad.w) * rho.cpu().numpy()))
    assert abs(charge - float(np.sum(w.occ))) < 1e-9 * float(np.sum(w.occ))
