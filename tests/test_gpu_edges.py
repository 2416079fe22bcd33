"""Edge cases on the GPU: the largest block (k = 64 right-hand sides, every
kernel shape at its widest), odd and single-column blocks, a mesh whose row
count fills no tile exactly, and argument errors on a live context."""
import numpy as np
import pytest
import scipy.sparse as sp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from ks_inputs import make_workload
from paper_2404_19249_amd.binding import KSError

DEV = "cuda:0"


def _ctx(w, **kw):
    from paper_2404_19249_amd import KSContext
    print(f"[case] {w.name} order={w.mesh.order} n={w.mesh.n} k={w.k} {kw}", flush=True)
    return KSContext.from_workload(w, **kw)


def _csr(ctx, which):
    rp, cl, vl = ctx.export_operator(which)
    return sp.csr_matrix((vl, cl, rp), shape=(ctx.N, ctx.N))


@pytest.mark.parametrize("k", [1, 7, 64])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_block_solve_widths_reach_tolerance(k, prec):
    """S X = B for seeded B of width k (1, odd, the maximum 64); the relative
    residual of every column is recomputed on the host from the exported S."""
    w = make_workload("small_molecule", n=5)            # N = 729: no tile size divides it
    ctx = _ctx(w, k_max=64, tol_solve=1e-10)
    psi, lam = ctx.initial_guess(w.k)
    ctx.assemble(psi, w.occ, want_fields=False)
    S = _csr(ctx, 0)
    rng = np.random.default_rng(100 + k)
    Bh = rng.standard_normal((ctx.N, k))
    Bd = torch.tensor(Bh, device=DEV)
    X, st = ctx.block_solve_rhs(Bd, precision=prec)
    Xh = X.cpu().numpy()
    rel = np.linalg.norm(Bh - S @ Xh, axis=0) / np.linalg.norm(Bh, axis=0)
    assert st["converged"]
    assert rel.max() <= 1e-10 * 1.0001, (k, prec, rel.max())


def test_live_context_rejects_bad_widths():
    w = make_workload("small_molecule", n=4)
    ctx = _ctx(w, k_max=8)
    psi, lam = ctx.initial_guess(w.k)
    ctx.assemble(psi, w.occ, want_fields=False)
    for k in (0, 9):
        Bd = torch.zeros(ctx.N, max(k, 1), dtype=torch.float64, device=DEV)[:, :k].contiguous()
        with pytest.raises(KSError) as e:
            ctx.block_solve_rhs(Bd)
        assert e.value.code == -1
    with pytest.raises(KSError):
        ctx.scf_run(psi, lam, w.occ, tol=0.0)


def _jacobi_pcg(S, b, m):
    """m iterations of Jacobi-preconditioned CG from x = 0, column by column
    (the textbook recurrences, FP64)."""
    d = S.diagonal()
    X = np.zeros_like(b)
    for c in range(b.shape[1]):
        x = np.zeros(b.shape[0])
        r = b[:, c].copy()
        z = r / d
        p = z.copy()
        rz = r @ z
        for _ in range(m):
            q = S @ p
            a = rz / (p @ q)
            x += a * p
            r -= a * q
            z = r / d
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
        X[:, c] = x
    return X


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
def test_block_solve_stops_at_iteration_limit(m):
    """A block PCG cut off after m iterations (odd and even m: the x update of
    an even iteration is deferred to the next) returns the m-th CG iterate."""
    w = make_workload("small_molecule", n=5)
    ctx = _ctx(w, k_max=8, tol_solve=1e-14, max_it_solve=m)
    psi, lam = ctx.initial_guess(w.k)
    ctx.assemble(psi, w.occ, want_fields=False)
    S = _csr(ctx, 0)
    rng = np.random.default_rng(7 + m)
    Bh = rng.standard_normal((ctx.N, 3))
    X, st = ctx.block_solve_rhs(torch.tensor(Bh, device=DEV), precision="fp64")
    ref = _jacobi_pcg(S, Bh, m)
    assert not st["converged"]
    err = np.abs(X.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err < 1e-11, (m, err)


def test_fp32_operator_copy_is_the_rounded_operator():
    """The mixed form's FP32 copy of S, whether written by the assembly of a
    mixed-precision step or made on demand before a mixed solve, is S rounded
    to FP32 value by value."""
    w = make_workload("small_molecule", n=5)
    ctx = _ctx(w, k_max=8)
    psi, lam = ctx.initial_guess(w.k)
    half = (ctx.nnz + 1) // 2
    lam, rep = ctx.scf_step(psi, lam, w.occ, precision="mixed")
    S = ctx.debug_buffer("S", ctx.nnz)
    S32 = ctx.debug_buffer("S32", half).view(torch.float32)[:ctx.nnz]
    assert torch.equal(S32, S.float())
    ctx.assemble(psi, w.occ, want_fields=False)
    with pytest.raises(KSError):
        ctx.debug_buffer("S32", half)
    ctx.block_solve(psi, lam, "mixed")
    S = ctx.debug_buffer("S", ctx.nnz)
    S32 = ctx.debug_buffer("S32", half).view(torch.float32)[:ctx.nnz]
    assert torch.equal(S32, S.float())


def test_stream_probe_reports_a_bandwidth_below_the_peak():
    """ks_stream_probe: a plain stream cannot exceed the 8 TB/s HBM peak
    (the buffers, 256 MiB each, are far larger than the caches), and bad
    arguments are refused."""
    from paper_2404_19249_amd import stream_probe, KSError
    for kind in ("read", "copy", "triad"):
        g = stream_probe(kind, 1 << 28, nontemporal=True, reps=3)
        assert 500.0 < g < 8000.0, (kind, g)
    with pytest.raises(KSError):
        stream_probe("read", 1024)


def test_autotune_cache_file(tmp_path):
    """ks_autotune_cached: a missing file is a miss that tunes and appends one
    entry (fp64, fp32 and Poisson lines) keyed by device, order, size class,
    nonzeros per row and k; a second context of the same workload hits it
    and ends with the same kernels without tuning; another k misses; an entry
    naming a row block that does not exist, and lines that do not parse, are
    skipped; a block solve with the cached kernels reaches its tolerance."""
    k = 8
    w = make_workload("mixed", n=12, order=2, k=k)
    path = tmp_path / "spmm_tune.txt"

    def fresh():
        c = _ctx(w, k_max=k, tol_solve=1e-10)
        psi, _ = c.initial_guess(k)
        c.assemble(psi, w.occ, want_fields=False)
        return c

    a = fresh()
    assert not a.autotune_cached(k, path, reps=2)
    f = [ln.split() for ln in path.read_text().splitlines()]
    assert [x[5] for x in f] == ["fp64", "fp32", "poisson"]
    assert [int(x[4]) for x in f] == [k, k, 1]
    assert all(len(x) == 10 and x[0].startswith("gfx") and x[1] == "2" for x in f)
    log2n = int(f[0][2])
    assert 2 ** log2n <= a.N < 2 ** (log2n + 1)
    cfg = a.spmm_config()
    for x, n in zip(f, ("fp64", "fp32", "poisson")):
        assert (int(x[6]), int(x[7]), int(x[8])) == (cfg[f"ng_{n}"], cfg[f"tile_{n}"],
                                                      cfg[f"tile_threads_{n}"]), (x, cfg)
        assert float(x[9]) > 0.0
    a.close()

    b = fresh()
    assert b.autotune_cached(k, path, reps=2)
    assert b.spmm_config() == cfg
    assert len(path.read_text().splitlines()) == 3
    assert not b.autotune_cached(4, path, reps=2)
    assert len(path.read_text().splitlines()) == 6
    assert b.autotune_cached(4, path, reps=2)

    bad = tmp_path / "bad.txt"
    bad_fp64 = f[0][:7] + ["77", "512", "0.1"]
    bad.write_text("not an entry\n" + " ".join(bad_fp64) + "\n" +
                   "\n".join(" ".join(x) for x in f[1:]) + "\n")
    assert not b.autotune_cached(k, bad, reps=2)
    assert len(bad.read_text().splitlines()) == 4 + 3
    assert b.autotune_cached(k, bad, reps=2)

    S = _csr(b, 0)
    rng = np.random.default_rng(11)
    Bh = rng.standard_normal((b.N, k))
    for prec in ("fp64", "mixed"):
        X, st = b.block_solve_rhs(torch.tensor(Bh, device=DEV), precision=prec)
        rel = np.linalg.norm(Bh - S @ X.cpu().numpy(), axis=0) / np.linalg.norm(Bh, axis=0)
        assert st["converged"] and rel.max() <= 1e-10 * 1.0001, (prec, rel.max())
    with pytest.raises(KSError):
        b.autotune_cached(k, "", reps=2)
    b.close()


@pytest.mark.parametrize("k", [8, 24])
def test_autotuned_kernels_agree_and_solve(k):
    """ks_autotune checks every SpMM-phase candidate (row kernels, halo
    tiles) against the first row kernel on a fixed block and never keeps one
    that disagrees: on a mesh where the tile forms are available none is
    rejected, and block solves with the chosen kernels reach the tolerance,
    residuals recomputed on the host."""
    w = make_workload("mixed", n=12, order=2, k=k)      # N = 12,167, two tile passes and more
    ctx = _ctx(w, k_max=k, tol_solve=1e-10)
    psi, lam = ctx.initial_guess(k)
    ctx.assemble(psi, w.occ, want_fields=False)
    rep = ctx.autotune(k, reps=2)
    print(rep)
    for n in ("fp64", "fp32", "poisson"):
        assert all(v != -2.0 for v in rep[f"row_ms_{n}"].values())
        assert all(v != -2.0 for v in rep[f"tile_ms_{n}"].values())
    assert rep["tile_ms_fp32"]["85x512"] > 0.0
    S = _csr(ctx, 0)
    rng = np.random.default_rng(7)
    Bh = rng.standard_normal((ctx.N, k))
    for prec in ("fp64", "mixed"):
        X, st = ctx.block_solve_rhs(torch.tensor(Bh, device=DEV), precision=prec)
        rel = np.linalg.norm(Bh - S @ X.cpu().numpy(), axis=0) / np.linalg.norm(Bh, axis=0)
        assert st["converged"] and rel.max() <= 1e-10 * 1.0001, (prec, rel.max())
    ctx.close()
