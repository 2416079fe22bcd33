"""Benchmark: block BVP solve of the augmented subspace step on one MI355X.

A step is one iteration of Algorithm 3 (assemble S from the density,
solve the N_occ boundary value problems, project onto the augmented space,
nonlinear inner iteration with the small eigensolve, energies) on the
"mixed" workload: 10 nuclei, 64^3 hexahedra -> P2 tetrahedra
(N = 2,048,383 unknowns), N_occ = 24, moved mesh.  The headline value is
DOF*RHS/s of the block BVP solve, measured with HIP events inside the timed
steps.  The timed solves run to a 1e-9 relative residual (inside the metric's
1e-8 bound: at 1e-8 the step's eigenvalues still move by up to ~2e-8 Ha, at
1e-9 they stay within 1e-8 Ha of a tightly solved step); both tolerances are
reported, in the FP64 and the mixed (FP32 PCG inside FP64 refinement) forms,
with the eigenvalue and energy errors of each.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision mixed|fp64]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF*RHS/s of block BVP solve to 1e-8 residual; mixed vs FP64; HBM GB/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmm_bytes(N, nnz, k, sv):
    """Algorithmic HBM bytes of one SpMM phase launch (q = S p with the p.q
    reduction): matrix values + column indices + row pointers, the gathered
    block p read once, q written once."""
    return nnz * (sv + 4) + 4 * (N + 1) + 2 * N * k * sv


def cg_iteration_bytes(N, nnz, k, sv):
    """Algorithmic bytes of one block-PCG iteration (three phases): SpMM
    (matrix, read p, write q), r update (read r, q, write r), x/p update
    (read x, p, r, write x, p): 10 [N][k] vector streams; diagonal read twice.
    (The solver applies the x update of two iterations in one pass, so it
    moves 9.5 streams on average.)"""
    return nnz * (sv + 4) + 4 * (N + 1) + 2 * N * sv + 10 * N * k * sv


def shift_leg(w, k, psi0, lam0, occ, lam_1, vmin, reps=2, max_it=4000):
    """The block solve at step 0 with the smaller shift mu' = -lambda_1 + 1
    (S - lambda_1 M + M: harder conditioning, more iterations), in both
    forms: iterations, time and the whole solve's algorithmic bandwidth.
    lambda_1 is a Ritz value, an upper bound of the operator's lowest
    eigenvalue, so S may come out indefinite (the FP64 PCG reports the
    breakdown).  Then mu' = -min_q V_eff,q + 1, which keeps S positive
    definite: x^T (1/2 K + M[V_eff]) x >= min V_eff x^T M x since K is
    semidefinite and the quadrature weights are positive."""
    from paper_2404_19249_amd import KSContext, KSError
    tried = []
    for basis, mu2 in (("-lambda_1 + 1", float(-lam_1 + 1.0)), ("-min V_eff + 1", float(-vmin + 1.0))):
        ctx = KSContext.from_workload(w, mu=mu2, tol_solve=1e-8, tol_inner=1e-8, tol_poisson=1e-10,
                                      max_it_solve=max_it)
        try:
            out = _shift_solves(ctx, k, psi0, lam0, occ, reps, max_it)
            out.update({"mu": mu2, "mu_basis": basis, "lambda_1": lam_1, "min_veff": vmin,
                        "indefinite": tried})
            return out
        except KSError as e:
            if e.code != -5:  # not a breakdown
                raise
            tried.append({"mu": mu2, "mu_basis": basis})
        finally:
            ctx.close()
    return {"error": "S indefinite", "indefinite": tried}


def _shift_solves(ctx, k, psi0, lam0, occ, reps, max_it):
    """Both forms of the step-0 block solve on one context: median time,
    iterations and algorithmic bandwidth."""
    import numpy as np
    N, nnz = ctx.N, ctx.nnz
    ctx.assemble(psi0, occ, want_fields=False)
    out = {}
    for prec in ("fp64", "mixed"):
        times, st = [], None
        for _ in range(reps):
            _, st = ctx.block_solve(psi0, lam0, prec)
            times.append(st["seconds"])
        t = float(np.median(times))
        its = int(max(st["iters"]))
        if prec == "fp64":
            sb = its * cg_iteration_bytes(N, nnz, k, 8)
        else:
            sb = its * cg_iteration_bytes(N, nnz, k, 4) + st["refinements"] * (nnz * 12 + 4 * (N + 1) + 3 * N * k * 8)
        out[prec] = {"dof_rhs_per_s": N * k / t, "ms": t * 1e3, "iters_max": its,
                     "refinements": st["refinements"], "converged": st["converged"],
                     "relres_max": float(max(st["relres"])), "solve_GBs": sb / t / 1e9,
                     "solve_frac_hbm": sb / t / 1e9 / HBM_PEAK_GBS}
    out["mixed_speedup"] = out["fp64"]["ms"] / out["mixed"]["ms"]
    return out


def phase_rooflines(ctx, k, reps=10, with_projection=True):
    """Per-phase device time (HIP events, ks_time_kernel) and throughput against
    the algorithmic bytes / flops of each phase (per unit of work as defined
    for the hot path): potential-matrix assembly (a4), density and LDA at the
    quadrature points (a2), projection onto the augmented basis (a6/a7) and
    its FP64 MFMA GEMM."""
    ne, nq, nl, nnz, N = ctx.n_elems, ctx.n_q, ctx.n_loc, ctx.nnz, ctx.N
    m = ctx.N_H + k
    out = {}
    ms = ctx.time_kernel(7, k, reps)
    b = ne * nq * 8 + ne * nl * 4 + 80 * ne + 8 * nnz
    f = 2 * ne * nq * nl * (nl + 1) // 2
    out["a4_potential_assembly"] = {"ms": ms, "GBs": b / ms / 1e6, "frac_hbm": b / ms / 1e6 / HBM_PEAK_GBS,
                                    "GFLOPs": f / ms / 1e6, "bytes": b, "flops": f}
    ms = ctx.time_kernel(8, k, reps)
    b = ctx.n_nodes * k * 8 + ne * nl * 4 + ne * nq * 8
    out["a2_density"] = {"ms": ms, "GBs": b / ms / 1e6, "frac_hbm": b / ms / 1e6 / HBM_PEAK_GBS, "bytes": b}
    ms = ctx.time_kernel(9, k, reps)
    b = 3 * ne * nq * 8
    out["a2_lda"] = {"ms": ms, "GBs": b / ms / 1e6, "frac_hbm": b / ms / 1e6 / HBM_PEAK_GBS, "bytes": b}
    if with_projection:
        # the unit of a6: the projection onto the m-column basis (its bytes and
        # flops as the dense formulation defines them), in the form the inner
        # iteration runs (coarse blocks from the ELL interpolation, T^T H T on
        # the matrix cores) and in the dense form
        b = 12 * nnz + 4 * (N + 1) + 8 * N * m
        f = 2 * nnz * m + 2 * N * m * m
        for key, which in (("a6_projection", 10), ("a6_projection_dense", 12)):
            ms = ctx.time_kernel(which, k, reps)
            out[key] = {"ms": ms, "m": m, "GBs": b / ms / 1e6, "frac_hbm": b / ms / 1e6 / HBM_PEAK_GBS,
                        "TFLOPs": f / ms / 1e9, "bytes": b, "flops": f}
        # MFMA fraction from the flops the kernel executes: 16x16 tiles on
        # and above the diagonal of the padded k x k product
        tb = (k + 15) // 16
        f_exec = 2 * N * 256 * tb * (tb + 1) // 2
        ms = ctx.time_kernel(11, k, reps)
        out["a6_gemm_mfma_f64"] = {"ms": ms, "executed_flops": f_exec, "TFLOPs": f_exec / ms / 1e9,
                                   "frac_mfma_f64": f_exec / ms / 1e9 / 78.6,
                                   "product": f"T^T (H T), N x {k}"}
    return out


def profiled_traffic(key):
    """HBM bytes per launch of the kernel configuration `key`, from the rocprofv3
    counter summaries committed under profiles/ (None if that configuration was
    not profiled)."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if line.startswith("traffic_bytes_per_launch ") and ":" in line:
                k, v = line[len("traffic_bytes_per_launch "):].rsplit(":", 1)
                if k.strip() == key:
                    return float(v)
    return None


def copy_probe(torch, nbytes=1 << 30, reps=10):
    """Device-to-device copy of 1 GiB with torch's plain copy kernel: read +
    write bytes per second (a practical HBM reference next to the 8 TB/s
    nominal peak)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def stream_probes(nbytes=1 << 32, reps=10):
    """Hand-written HBM streaming probes (ks_stream_probe, nontemporal
    16-byte vector streams): read, copy and triad bandwidth, and the write
    bandwidth implied by read and copy (a copy moves one read and one write
    stream: 2 / copy = 1 / read + 1 / write)."""
    from paper_2404_19249_amd import stream_probe
    out = {kind: stream_probe(kind, nbytes, nontemporal=True, reps=reps) for kind in ("read", "copy", "triad")}
    inv_w = 2.0 / out["copy"] - 1.0 / out["read"]
    out["write_implied"] = 1.0 / inv_w if inv_w > 0 else None
    out["buffer_bytes"] = nbytes
    return out


def mix_ceiling(probes, read_bytes, write_bytes):
    """Streaming ceiling (GB/s) for a kernel that reads read_bytes and writes
    write_bytes: the time of those streams at the probes' read and implied
    write bandwidth."""
    if not probes.get("write_implied"):
        return probes["copy"]
    t = read_bytes / probes["read"] + write_bytes / probes["write_implied"]
    return (read_bytes + write_bytes) / t


def cpu_info():
    """CPU model and logical CPU count of this host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(k, tol, n=24, n_inner=None, N_full=None):
    """The oracle, single thread, on a bounded sample of the same workload:
    the mixed workload's nuclei and mesh recipe at n^3 hexahedra (n = 24:
    N = 103,823), the BVP operator S = 1/2 K + M[V_ext + V_H + V_xc] + mu M
    of the initial guess's density (Hartree and LDA included, as on the
    GPU).  Timed legs: the assembly of S, the block solve of the k BVPs to
    `tol` (the value), one projection (F_B, F_A^L) and one inner iteration
    (Poisson, LDA, M[V_nl], its projection, the small eigensolve, the new
    density).  The whole step at full size is extrapolated from these legs,
    linear in N, with the GPU step's inner iteration count."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from ks_inputs import make_workload
    from oracle.step import KSProblem, initial_guess, block_solve, small_eig
    from oracle.xc import lda_xc
    w = make_workload("mixed", n=n, k=k)
    legs = {}
    with threadpool_limits(1):
        p = KSProblem.from_workload(w)
        th, Psi = initial_guess(p, w.k)
        rho = p.density(Psi)
        wB = p.boundary_data(rho)
        VH, _ = p.hartree_nodes(rho, wB, 1e-10)
        t0 = time.perf_counter()
        _, vxc = lda_xc(rho, p.xc_mode)
        veff = p.vext_q + p.at_quad(VH) + vxc
        S = (0.5 * p.K_II + p.potential_matrix(veff) + p.mu * p.M_II).tocsr()
        legs["assembly_s"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        X, its, rr = block_solve(p, S, Psi, th, tol=tol)
        dt = time.perf_counter() - t0
        legs["block_solve_s"] = dt
        t0 = time.perf_counter()
        G = p.P.T @ (p.M_II @ p.P)
        T = np.linalg.solve(G, p.P.T @ (p.M_II @ X))
        Z = np.hstack([p.P, X - p.P @ T])
        FB = Z.T @ (p.M_II @ Z)
        FAL = Z.T @ (p.A_linear() @ Z)
        legs["projection_s"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        VHi, _ = p.hartree_nodes(rho, wB, 1e-12)
        _, vx = lda_xc(rho, p.xc_mode)
        FA = FAL + Z.T @ (p.potential_matrix(p.at_quad(VHi) + vx) @ Z)
        _, U, _, _ = small_eig(FA, FB, w.k)
        p.density(Z @ U)
        legs["inner_iteration_s"] = time.perf_counter() - t0
    model, nproc = cpu_info()
    out = {"value": p.N * w.k / dt, "unit": "DOF*RHS/s", "cores": 1, "kind": "oracle",
           "sample": f"mixed workload recipe at {n}^3 hexes P2 (N={p.N}, k={w.k}, nnz={p.K_II.nnz}),"
                     f" S with Hartree and LDA from the initial guess's density: one FP64 block"
                     f" Jacobi-PCG solve to {tol:g}, {int(max(its))} iterations, {dt:.2f} s",
           "cpu_model": model, "nproc": nproc, "legs": legs, "N": int(p.N)}
    if n_inner and N_full:
        per = legs["assembly_s"] + legs["block_solve_s"] + legs["projection_s"] + n_inner * legs["inner_iteration_s"]
        out["step_extrapolated_s"] = per * N_full / p.N
        out["step_extrapolation"] = (f"(assembly + solve + projection + {n_inner} inner iterations) at N={p.N},"
                                     f" scaled linearly to N={N_full}")
    return out


def batched_leg(torch, np, reps=3):
    """The batched workload: 48 independent systems of uneven size (P1/P2,
    12^3..40^3 hexes, k = 1..12) solved together in one persistent launch
    replayed from a hipGraph, after the layout autotuner; against the same
    systems solved one after another with the single-system solver."""
    from ks_inputs.workloads import batched_systems
    from paper_2404_19249_amd import KSContext, KSBatch
    t0 = time.perf_counter()
    ws = batched_systems(48)
    ctxs, psis, lams = [], [], []
    for w in ws:
        c = KSContext.from_workload(w, tol_solve=1e-8, tol_inner=1e-8, tol_poisson=1e-10)
        psi, lam = c.initial_guess(w.k)
        c.assemble(psi, w.occ, want_fields=False)
        ctxs.append(c); psis.append(psi); lams.append(lam)
    setup = time.perf_counter() - t0
    seq = []
    for c, p, l in zip(ctxs, psis, lams):
        c.block_solve(p, l)
    for c, p, l in zip(ctxs, psis, lams):
        seq.append(c.block_solve(p, l)[1]["seconds"])
    b = KSBatch(ctxs, [w.k for w in ws])
    tuned_ms = b.autotune(psis, lams, rounds=4)
    launches, st = [], None
    for r in range(reps):
        outs, st = b.block_solve(psis, lams)
        launches.append(st["seconds"])
    t = float(np.median(launches))
    ss = np.array(st["system_seconds"]) * 1e3
    dofs = sum(c.N * w.k for c, w in zip(ctxs, ws))
    its = st["iters"]
    byt = sum(i * cg_iteration_bytes(c.N, c.nnz, w.k, 8) for i, c, w in zip(its, ctxs, ws))
    out = {"systems": len(ws), "sum_N_k": dofs, "launch_ms": t * 1e3,
           "dof_rhs_per_s": dofs / t, "p50_system_ms": float(np.percentile(ss, 50)),
           "p99_system_ms": float(np.percentile(ss, 99)), "max_system_ms": float(ss.max()),
           "sequential_device_ms": sum(seq) * 1e3, "speedup_vs_sequential": sum(seq) / t,
           "grid": b.grid, "autotune_best_ms": tuned_ms,
           "tiled_systems": sum(1 for x in b.tile if x),
           "iteration_GBs": byt / t / 1e9, "relres_max": float(max(st["relres"])),
           "setup_s": setup}
    b.close()
    for c in ctxs:
        c.close()
    return out


def scf_run_leg(np, w, precision, tol=2e-4, max_steps=60):
    """Algorithm 3 run to convergence on the bench workload: from the coarse
    Ritz initial guess, steps until the density changes by less than tol in
    the quadrature L2 norm (the tolerance Sec. 4 sets for Algorithm 3); wall
    time of the whole run, step count, E_total and E_KS of the last step."""
    import torch
    from paper_2404_19249_amd import KSContext
    ctx = KSContext.from_workload(w, tol_solve=1e-8, tol_inner=1e-8, tol_poisson=1e-10)
    psi, lam = ctx.initial_guess(w.k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lam, rep = ctx.scf_run(psi, lam, w.occ, tol=tol, max_steps=max_steps, precision=precision)
    torch.cuda.synchronize()
    out = dict(rep)
    out["wall_s"] = time.perf_counter() - t0
    out["tol"] = tol
    out["lambda"] = [float(x) for x in lam[:4]]
    ctx.close()
    return out


COMPARE_SIZES = {"lih": (12, 14, 16, 20, 24, 28, 34, 44), "ch4": (12, 14, 16, 20, 26, 34, 44, 56),
                 "c6h6": (14, 16, 20, 24, 32, 44, 56)}


def compare_leg(np, molecules=("lih", "ch4", "c6h6"), k_asm=4, tol=2e-4, max_steps=300, precision="mixed"):
    """Algorithm 3 against the direct method along a mesh sequence, as
    Algorithm 2 runs them (Sec. 3.3; Sec. 4, Tables 1-3: LiH, CH4, C6H6 in
    (-10, 10)^3, P1 elements, cumulative time against the element count).

    The meshes are n^3 hexahedra moved toward the nuclei for the n in
    COMPARE_SIZES (1.0e4 .. 1.1e6 elements; the paper's tables span 9e3 ..
    2.8e6); a mesh is not adapted to the density.  Level 1 starts from the
    coarse Ritz guess; every later level starts from the previous level's
    orbitals carried over by Algorithm 1 (ks_interpolate, then
    M-orthonormalised) and its eigenvalues.  The first k_asm levels use the
    direct SCF (Algorithm 2's threshold K_asm = 4); after them three chains
    go on from the same state: the direct SCF (LOBPCG to a relative residual
    of 1e-6), Algorithm 3 with the paper's shift mu = 8 M sum Z^2, and
    Algorithm 3 with mu = 2 (1 - lambda_1) from the previous level's lowest
    eigenvalue (H~ + mu M stays positive definite while lambda_1 moves by less
    than 1 - lambda_1); BVPs to 1e-8, each until the density changes by less
    than tol.  Per level: element count, iterations, seconds (interpolation
    included, mesh set-up not), E_total; the cumulative seconds of each
    chain."""
    import torch
    from ks_inputs import make_workload
    from paper_2404_19249_amd import KSContext
    chains = ("direct", "algorithm3", "algorithm3_small_mu")
    out = {"tol": tol, "k_asm": k_asm, "precision": precision, "molecules": []}
    for name in molecules:
        carry = dict.fromkeys(chains)
        cum = dict.fromkeys(chains, 0.0)
        levels = []
        for lev, n in enumerate(COMPARE_SIZES[name]):
            w = make_workload(name, n=n)
            row = {"level": lev + 1, "n": n}
            for method in (("direct",) if lev < k_asm else chains):
                prev = carry[method]
                mu = None
                if method == "algorithm3_small_mu":
                    mu = 2.0 * (1.0 - float(prev[2][0]))
                ctx = KSContext.from_workload(w, mu=mu, tol_solve=1e-8, tol_inner=1e-8, tol_poisson=1e-10)
                row.update(elements=ctx.n_elems, N=ctx.N)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if prev is None:
                    psi, lam = ctx.initial_guess(w.k)
                else:
                    psi = ctx.interpolate(prev[0], prev[1], orthonormalize=True)
                    lam = prev[2].copy()
                if method == "direct":
                    lam, rep = ctx.direct_scf(psi, lam, w.occ, tol=tol, max_scf=max_steps, tol_eig=1e-6,
                                              max_eig=3000)
                    it = {"scf_iters": rep["scf_iters"], "eig_iters": rep["eig_iters"]}
                else:
                    lam, rep = ctx.scf_run(psi, lam, w.occ, tol=tol, max_steps=max_steps, precision=precision)
                    it = {"steps": rep["steps"], "inner_iters": rep["inner_iters"], "mu": ctx.mu}
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                ctx.close()
                row[method] = dict(it, seconds=dt, converged=bool(rep["converged"]), E_total=rep["E_total"],
                                   lambda_1=float(lam[0]))
                if lev < k_asm:
                    for ch in chains:
                        carry[ch] = (w.mesh, psi, lam)
                        cum[ch] += dt
                else:
                    carry[method] = (w.mesh, psi, lam)
                    cum[method] += dt
            row["cumulative_s"] = dict(cum)
            log(f"[bench] compare {name} {json.dumps(row)}")
            levels.append(row)
        out["molecules"].append({"molecule": name, "k": w.k, "levels": levels})
    return out


def adaptive_leg(np, name="lih", sizes=(12, 16, 20, 24, 28, 34), eps=1e-3, h_min=0.25, h_max=2.0, omega=0.8,
                 sweeps=20, tol=1e-6):
    """Algorithm 2's mesh moving (Sec. 3.2) against fixed meshes of the same
    size: on every level, the direct SCF (to a density change below tol) on
    (a) the uniform Kuhn mesh of the box, (b) the mesh moved toward the
    nuclei by the fixed map of the workloads, (c) the r-adapted mesh: the
    previous level's displacement (moved minus uniform node positions) is
    carried to the new uniform lattice (ks_interpolate_field over the
    previous uniform lattice; the uniform lattice itself if that would
    invert an element), then moved by `sweeps` spring sweeps under the metric
    of sqrt(rho) of the previous level's solution (ks_mesh_metric on its own
    mesh, carried to the new nodes by ks_interpolate_field, ks_move_nodes);
    its orbitals carried over by Algorithm 1.  With the same number of
    unknowns, a lower E_total is the better mesh (the discrete problem is a
    Ritz-Galerkin approximation).  Level 1 of (c) is the uniform mesh."""
    import dataclasses
    import torch
    from ks_inputs import make_workload
    from ks_inputs.mesh import freudenthal_mesh
    from paper_2404_19249_amd import KSContext, mesh_metric, move_nodes, interpolate_field
    rows, prev, prev_lat, prev_disp = [], None, None, None

    def min_det(x, el):
        X = x[el[:, :4]]
        J = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)
        return float(np.linalg.det(J).min())

    for lev, n in enumerate(sizes):
        w = make_workload(name, n=n)
        lattice = freudenthal_mesh(n, w.mesh.L, 1)
        row = {"level": lev + 1, "n": n, "elements": int(lattice.n_elems)}
        meshes = {"uniform": lattice, "moved_to_nuclei": w.mesh}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if prev is None:
            meshes["metric_moved"] = lattice
        else:
            pm, ppsi, _ = prev
            start = lattice.coords
            d = interpolate_field(prev_lat, torch.tensor(prev_disp, device="cuda"), lattice.coords).cpu().numpy()
            if min_det(lattice.coords + d, lattice.elems) > 0.0:
                start = lattice.coords + d
            row["carried_displacement"] = start is not lattice.coords
            M = mesh_metric(pm, ppsi, w.occ, eps, h_min, h_max)
            Mn = interpolate_field(pm, M, start)
            xs, hv = move_nodes(dataclasses.replace(lattice, coords=start), Mn, omega=omega, sweeps=sweeps)
            meshes["metric_moved"] = dataclasses.replace(lattice, coords=xs, moved=True)
            row["move_halvings"] = hv
        torch.cuda.synchronize()
        row["metric_and_move_s"] = time.perf_counter() - t0
        for key, mesh in meshes.items():
            wk = dataclasses.replace(w, mesh=mesh)
            ctx = KSContext.from_workload(wk, tol_solve=1e-8, tol_inner=1e-8, tol_poisson=1e-10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if key == "metric_moved" and prev is not None:
                psi = ctx.interpolate(prev[0], prev[1], orthonormalize=True)
                lam = prev[2].copy()
            else:
                psi, lam = ctx.initial_guess(w.k)
            lam, rep = ctx.direct_scf(psi, lam, w.occ, tol=tol, max_scf=300, tol_eig=1e-8, max_eig=4000)
            torch.cuda.synchronize()
            row[key] = {"E_total": rep["E_total"], "lambda_1": float(lam[0]), "scf_iters": rep["scf_iters"],
                        "converged": bool(rep["converged"]), "seconds": time.perf_counter() - t0}
            if key == "metric_moved":
                prev = (mesh, psi, lam)
            ctx.close()
        prev_lat, prev_disp = lattice, meshes["metric_moved"].coords - lattice.coords
        log(f"[bench] adaptive {name} h_min={h_min} sweeps={sweeps} n={n}: " + ", ".join(
            f"{key} {row[key]['E_total']:.5f}" for key in meshes) + f"; halvings {row.get('move_halvings', 0)}")
        rows.append(row)
    return {"molecule": name, "eps": eps, "h_min": h_min, "h_max": h_max, "omega": omega, "sweeps": sweeps,
            "tol": tol, "levels": rows}


def differentiation_leg(np, warm_steps=2, atom=0, axis=0, h=1e-4):
    """The differentiation workload: 20 nuclei, 96^3 hexes -> P1 tetrahedra
    (N = 857,375), N_occ = 40.  One step forward (with E_KS) and its adjoint
    backward (dE/dV_ext at the quadrature points and the nuclear forces),
    timed; the force on one nuclear coordinate is checked against a central
    finite difference of E_KS with step h (Bohr), both steps started from the
    same orbitals."""
    import torch
    from ks_inputs import make_workload
    from paper_2404_19249_amd import KSContext
    w = make_workload("differentiation")
    ctx = KSContext.from_workload(w, tol_solve=1e-11, tol_inner=1e-11, tol_poisson=1e-12,
                                  max_it_inner=80)
    psi, lam = ctx.initial_guess(w.k)
    for i in range(warm_steps):
        lam, rep = ctx.scf_step(psi, lam, w.occ)
        log(f"[bench] differentiation warm step {i}: inner {rep['inner_iters']} "
            f"{rep['seconds'][5]:.2f}s")
    psi0, lam0 = psi.clone(), lam.copy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = psi0.clone()
    _, rep = ctx.scf_step(p, lam0, w.occ)
    e = ctx.step_energy()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g, F, st = ctx.step_backward(dE=1.0, want_forces=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    R0 = np.array(w.atoms.R, dtype=np.float64)
    # mesh-motion (Pulay) terms: nodes follow the nuclei with Gaussian weights
    d2 = np.sum((np.asarray(w.mesh.coords)[:, None, :] - R0[None, :, :]) ** 2, axis=-1)
    motion = torch.tensor(np.exp(-d2 / 4.0), device="cuda")
    del d2
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    dX, _, Fm, st_m = ctx.step_backward_mesh(dE=1.0, motion=motion)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    del motion
    pulay = {"mesh_backward_s": t4 - t3, "motion": "Gaussian weights exp(-|x - R_a|^2 / 4)",
             "max_abs_dE_dX": float(dX.abs().max()),
             "mesh_term_over_fixed_mesh_force": float(np.abs(Fm - F).max() / np.abs(F).max())}
    del dX
    # reverse mode through the truncated FP64 PCG of the same step (checkpoints
    # every 8 iterations), against the implicit adjoint
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    g_t, F_t, st_t = ctx.step_backward(dE=1.0, want_forces=True, truncated=True, seg=8)
    torch.cuda.synchronize()
    t6 = time.perf_counter()
    truncated = {"backward_s": t6 - t5, "seg": 8, "solve_iters_max": int(max(st_t["iters"][:w.k])),
                 "force_rel_diff_vs_implicit": float(np.abs(F_t - F).max() / np.abs(F).max()),
                 "grad_rel_diff_vs_implicit": float((g_t - g).abs().max() / g.abs().max())}
    del g_t
    E = []
    for sgn in (1, -1):
        R = R0.copy()
        R[atom, axis] += sgn * h
        ctx.set_external(R=R)
        p = psi0.clone()
        ctx.scf_step(p, lam0, w.occ)
        E.append(ctx.step_energy()["KS"])
    ctx.set_external(R=R0)
    f_fd = -(E[0] - E[1]) / (2 * h)
    f_adj = float(F[atom, axis])
    out = {"N": ctx.N, "k": w.k, "n_atoms": int(len(R0)), "forward_step_s": t1 - t0,
           "backward_s": t2 - t1, "backward_over_forward": (t2 - t1) / (t1 - t0),
           "adjoint_solve_iters_max": int(max(st["iters"][:w.k])),
           "E_KS": e["KS"], "status": rep["status"], "inner_iters": rep["inner_iters"],
           "res_inner": rep["res_inner"], "adjoint_converged": bool(st["converged"]),
           "force_check": {"atom": atom, "axis": axis, "h": h, "adjoint": f_adj, "central_fd": f_fd,
                           "rel_err": abs(f_adj - f_fd) / max(abs(f_fd), 1e-300)},
           "grad_q_values": int(g.numel()), "pulay": pulay, "truncated_reverse": truncated}
    ctx.close()
    return out


def solve_forms(ctx, k, psi, lam, occ, tols, reps=5):
    """Both forms of the block solve on the operator assembled from psi, at
    each tolerance: median device time, iterations, refinements, final
    relative residual and the whole solve's algorithmic bandwidth."""
    import numpy as np
    N, nnz = ctx.N, ctx.nnz
    ctx.assemble(psi, occ, want_fields=False)
    out = {}
    for tol in tols:
        ctx.set_options(tol_solve=tol)
        res = {}
        for prec in ("fp64", "mixed"):
            times, st = [], None
            for _ in range(reps):
                _, st = ctx.block_solve(psi, lam, prec)
                times.append(st["seconds"])
            t = float(np.median(times))
            its = int(max(st["iters"]))
            # whole-solve algorithmic bytes: iterations x B_it (+ the FP64
            # residual SpMMs b - S x of the refinement loop in the mixed form)
            if prec == "fp64":
                sb = its * cg_iteration_bytes(N, nnz, k, 8)
            else:
                sb = its * cg_iteration_bytes(N, nnz, k, 4) + st["refinements"] * (nnz * 12 + 4 * (N + 1) + 3 * N * k * 8)
            res[prec] = {"dof_rhs_per_s": N * k / t, "ms": t * 1e3, "iters_max": its,
                         "refinements": st["refinements"], "converged": bool(st["converged"]),
                         "relres_max": float(max(st["relres"])),
                         "solve_GBs": sb / t / 1e9, "solve_frac_hbm": sb / t / 1e9 / HBM_PEAK_GBS}
        res["mixed_speedup"] = res["fp64"]["ms"] / res["mixed"]["ms"]
        # O'Leary's block CG (FP64, one Krylov block): fewer iterations,
        # each with two k x k Gram products and two block updates more
        times, st = [], None
        for _ in range(max(1, reps // 2)):
            _, st = ctx.block_solve(psi, lam, "block_cg")
            times.append(st["seconds"])
        t = float(np.median(times))
        res["fp64_block_cg"] = {"ms": t * 1e3, "iters_max": int(max(st["iters"])),
                                "converged": bool(st["converged"]), "relres_max": float(max(st["relres"])),
                                "over_fp64_per_column": t * 1e3 / res["fp64"]["ms"]}
        out[f"tol_{tol:g}"] = res
    return out


def eig_accuracy(w, ctx, psi, lam, occ, tols):
    """Eigenvalues and E_total of one step from (psi, lam) in each form and
    at each solve tolerance against the same step with the BVPs solved to
    1e-12 in FP64; all inner iterations to 1e-11.  Every step's status is
    kept: an error is only meaningful when both steps converged."""
    import numpy as np
    from paper_2404_19249_amd import KSContext
    ref_ctx = KSContext.from_workload(w, tol_solve=1e-12, tol_inner=1e-11, tol_poisson=1e-12,
                                      max_it_inner=100)
    lam_ref, rr = ref_ctx.scf_step(psi.clone(), lam, occ, precision="fp64")
    ref_ctx.close()
    out = {"reference": {"status": rr["status"], "inner_iters": rr["inner_iters"],
                         "res_inner": rr["res_inner"], "solve_iters_max": int(max(rr["solve"]["iters"])),
                         "tol_solve": 1e-12, "tol_inner": 1e-11}}
    for tol in tols:
        ctx.set_options(tol_solve=tol, tol_inner=1e-11, tol_poisson=1e-12, max_it_inner=100)
        for prec in ("fp64", "mixed"):
            l2, r2 = ctx.scf_step(psi.clone(), lam, occ, precision=prec)
            out[f"{prec}_tol_{tol:g}"] = {
                "status": r2["status"], "res_inner": r2["res_inner"],
                "relres_max": float(max(r2["solve"]["relres"])),
                "eig_err_Ha": float(np.abs(l2 - lam_ref).max()),
                "E_total_err_Ha": abs(r2["E_total"] - rr["E_total"]),
                "both_converged": rr["status"] == 0 and r2["status"] == 0}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol-solve", type=float, default=1e-9,
                    help="relative residual of the timed block solves (the metric's bound is 1e-8; "
                         "1e-9 keeps every eigenvalue of the step within 1e-8 Ha)")
    ap.add_argument("--no-shift-leg", action="store_true",
                    help="skip the secondary solve with mu' = -lambda_1 + 1")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--workload", default="mixed")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form leg")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default SpMM kernels (for profiling one configuration)")
    ap.add_argument("--no-differentiation", action="store_true",
                    help="skip the differentiation workload (forward + adjoint, FD check)")
    ap.add_argument("--compare", action="store_true",
                    help="also run Algorithm 3 against the direct SCF along a mesh sequence on "
                         "the paper's molecules (LiH, CH4, C6H6)")
    ap.add_argument("--scf-run", action="store_true",
                    help="also run Algorithm 3 to convergence (density change < 2e-4) from the "
                         "coarse initial guess on the bench workload")
    ap.add_argument("--mode", default="step", choices=["step", "solve", "compare", "adaptive"],
                    help="solve: skip the SCF steps (block solves and kernel timings only, "
                         "for profiling); compare: only the mesh-sequence comparison; adaptive: "
                         "only the metric-moved mesh sequence against fixed meshes")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the sharded "
              "multi-GPU path is design only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from ks_inputs import make_workload
    from paper_2404_19249_amd import KSContext

    if args.mode == "compare":
        print(json.dumps({"compare": compare_leg(np)}), flush=True)
        return
    if args.mode == "adaptive":
        runs = []
        for name in ("lih", "ch4"):
            runs.append(adaptive_leg(np, name))
        print(json.dumps({"adaptive": runs}), flush=True)
        return
    t_setup = time.perf_counter()
    w = make_workload(args.workload, n=args.n)
    k = w.k
    tol = args.tol_solve
    ctx = KSContext.from_workload(w, tol_solve=tol, tol_inner=1e-8, tol_poisson=1e-10)
    N, nnz = ctx.N, ctx.nnz
    log(f"[bench] {w.name}: N={N} nnz={nnz} k={k} colours={ctx.n_colours} mu={ctx.mu:.1f} "
        f"setup {time.perf_counter() - t_setup:.1f}s")
    occ = w.occ
    psi0, lam0 = ctx.initial_guess(k)
    copy_gbs = copy_probe(torch)
    probes = stream_probes()
    log(f"[bench] device copy probe (torch): {copy_gbs:.0f} GB/s; streaming probes: {json.dumps(probes)}")
    ctx.assemble(psi0, occ, want_fields=False)
    tune = None if args.no_autotune else ctx.autotune(k, reps=10)
    log(f"[bench] autotune: {json.dumps(tune)}")
    if args.mode == "solve":
        args.warmup, args.steps = 0, 0
    # The timed state: one step from the coarse Ritz guess (step 0).  From the
    # guess itself the inner iteration does not converge on this workload
    # (the augmented space's gap at the 24th level is a few mHa and the
    # Anderson iteration oscillates, as the oracle's does on the 32^3 mesh),
    # so every timed step starts from the state after it, where it converges.
    psi1, lam1 = psi0.clone(), lam0.copy()
    lam1, rep0 = ctx.scf_step(psi1, lam1, occ, precision=args.precision)
    step0 = {"status": rep0["status"], "inner_iters": rep0["inner_iters"], "res_inner": rep0["res_inner"],
             "solve_iters_max": int(max(rep0["solve"]["iters"])), "seconds": rep0["seconds"][5]}
    log(f"[bench] step 0 (prepares the timed state): {json.dumps(step0)}")
    psi = psi1.clone()
    for i in range(args.warmup):
        psi.copy_(psi1)
        lam, rep = ctx.scf_step(psi, lam1.copy(), occ, precision=args.precision)
        log(f"[bench] warmup step {i}: status {rep['status']} inner {rep['inner_iters']} solve iters "
            f"{max(rep['solve']['iters'])} {rep['seconds'][5]:.3f}s")
    # ------------------------------------------------------------ timed steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solve_s, reps = 0.0, []
    for i in range(args.steps):
        psi.copy_(psi1)   # one pass of the step over the same input state
        lam, rep = ctx.scf_step(psi, lam1.copy(), occ, precision=args.precision)
        solve_s += rep["solve"]["seconds"]
        reps.append(rep)
        log(f"[bench] step {i}: status={rep['status']} E={rep['E_total']:.8f} inner={rep['inner_iters']} "
            f"solve={rep['solve']['seconds'] * 1e3:.2f}ms iters={max(rep['solve']['iters'])} "
            f"refine={rep['solve']['refinements']} res_inner={rep['res_inner']:.2e} total={rep['seconds'][5]:.3f}s")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / max(args.steps, 1)
    value = N * k * args.steps / solve_s if args.steps else None
    # per-phase rooflines on the state the last step left (assembly, fields, projection)
    phases_other = phase_rooflines(ctx, k, with_projection=args.steps > 0)
    log(f"[bench] phases: {json.dumps(phases_other)}")

    # ------------------------------------- both forms on the same inputs
    tols = sorted({tol, 1e-8})
    forms = solve_forms(ctx, k, psi1, lam1, occ, tols)
    forms["state"] = "after one step from the coarse Ritz guess (the timed steps' input)"
    forms["step0_state"] = solve_forms(ctx, k, psi0, lam0, occ, tols)
    ctx.set_options(tol_solve=tol, tol_inner=1e-8, tol_poisson=1e-10, max_it_inner=50)
    if value is None:
        value = forms[f"tol_{tol:g}"][args.precision]["dof_rhs_per_s"]
    if args.mode == "step":
        forms["eig_accuracy"] = eig_accuracy(w, ctx, psi1, lam1, occ, tols)
        log(f"[bench] eigenvalue accuracy: {json.dumps(forms['eig_accuracy'])}")
        ctx.set_options(tol_solve=tol, tol_inner=1e-8, tol_poisson=1e-10, max_it_inner=50)

    # ------------------------------------------- roofline of the SpMM phase
    ctx.assemble(psi1, occ, want_fields=False)
    ctx.block_solve(psi1, lam1, "mixed")   # leaves the FP32 operator and workspace
    sv = 4 if args.precision == "mixed" else 8
    which = 3 if args.precision == "mixed" else 0
    ms_a = ctx.time_kernel(which, k, args.reps)
    ms_b = ctx.time_kernel(which + 1, k, args.reps)
    ms_c = ctx.time_kernel(which + 2, k, args.reps)
    ms_a64 = ctx.time_kernel(0, k, args.reps)
    bytes_a = spmm_bytes(N, nnz, k, sv)
    ach = bytes_a / (ms_a * 1e-3) / 1e9
    cfg = ctx.spmm_config()
    tile = cfg["tile_fp32" if sv == 4 else "tile_fp64"]
    tname = "float" if sv == 4 else "double"
    if tile > 0:
        tb = cfg["tile_threads_fp32" if sv == 4 else "tile_threads_fp64"]
        kname = f"k_tpcg_A<{tname},{16 // sv},16,{tb}>"
        kdesc = f"k_tpcg_A<{tname}> halo-tile SpMM, {tile}-row blocks, {tb} threads (q = S p, p.q), k={k}"
    else:
        kname, kdesc = f"k_pcg_A<{tname}>", f"k_pcg_A<{tname}> row kernel (q = S p, p.q), k={k}"
    traffic = profiled_traffic(f"{kname} tile={tile} N={N} k={k}")
    roof = {"kernel": kdesc, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS,
            "traffic": None if traffic is None else traffic / 1e9,
            "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE)",
            "bytes_per_launch": bytes_a, "ms_per_launch": ms_a, "spmm_config": cfg,
            # against the streaming ceiling for this kernel's read/write mix (hand-written
            # probes of the same run), against torch's copy, and algorithmic / measured bytes
            "probe_ceiling_GBs": mix_ceiling(probes, bytes_a - N * k * sv, N * k * sv),
            "frac_probe": ach / mix_ceiling(probes, bytes_a - N * k * sv, N * k * sv),
            "frac_torch_copy": ach / copy_gbs,
            "algorithmic_over_traffic": None if not traffic else bytes_a / traffic}
    it_bytes = cg_iteration_bytes(N, nnz, k, sv)
    it_gbs = it_bytes / ((ms_a + ms_b + ms_c) * 1e-3) / 1e9
    phases = {"spmm_ms": ms_a, "r_update_ms": ms_b, "xp_update_ms": ms_c,
              "iteration_GBs": it_gbs, "iteration_frac_probe": it_gbs / copy_gbs,
              "fp64_spmm_ms": ms_a64,
              "fp64_spmm_GBs": spmm_bytes(N, nnz, k, 8) / (ms_a64 * 1e-3) / 1e9}
    for ph in phases_other.values():
        if "GBs" in ph:
            ph["frac_probe"] = ph["GBs"] / copy_gbs
    for key, res in forms.items():
        if key.startswith("tol_"):
            for prec in ("fp64", "mixed"):
                res[prec]["solve_frac_probe"] = res[prec]["solve_GBs"] / copy_gbs
    statuses = [r["status"] for r in reps]
    out = {
        "metric": METRIC, "value": value, "unit": "DOF*RHS/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.atoms.M} nuclei, {w.mesh.n}^3 hexes P{w.mesh.order} "
                               f"tets, moved mesh, N={N}, k={k}, nnz={nnz}",
                   "N": N, "k": k, "nnz": nnz, "precision": args.precision, "mu": ctx.mu,
                   "tol_solve": tol, "tol_inner": 1e-8,
                   "value_basis": "N*k / device time of the block solve inside each timed step "
                                   "(every step from the state after one step from the coarse "
                                   "Ritz guess)"},
        "roofline": roof,
        "copy_probe_GBs": copy_gbs,
        "stream_probes_GBs": probes,
        "autotune": tune,
        "pcg_phases": phases,
        "phases": phases_other,
        "block_solve": forms,
        "step0": step0,
        "step": {} if not reps else {
            "dof_rhs_per_s": N * k / (ms_per_step * 1e-3),
            "status": statuses, "all_converged": all(s == 0 for s in statuses),
            "res_inner": [r["res_inner"] for r in reps],
            "inner_iters": [r["inner_iters"] for r in reps],
            "solve_iters_max": [int(max(r["solve"]["iters"])) for r in reps],
            "solve_relres_max": [float(max(r["solve"]["relres"])) for r in reps],
            "poisson_iters": [r["poisson_iters"] for r in reps],
            "seconds_split": {n: float(np.mean([r["seconds"][i] for r in reps]))
                              for i, n in enumerate(["assemble", "solve", "project", "inner",
                                                     "energies", "total"])}},
    }
    vmin = None
    if not args.no_shift_leg and args.mode == "step":
        vmin = float(ctx.assemble(psi0, occ, want_fields=True)["veff_q"].min())
    ctx.close()
    if vmin is not None:
        log("[bench] secondary shift mu' = -lambda_1 + 1 ...")
        try:
            forms["shift_lambda1"] = shift_leg(w, k, psi0, lam0, occ, float(lam1[0]), vmin)
            log(f"[bench] shift leg: {json.dumps(forms['shift_lambda1'])}")
        except Exception as e:  # reported, never hides the headline
            forms["shift_lambda1"] = {"error": repr(e)}
    if not args.no_batched:
        log("[bench] batched form ...")
        try:
            forms["batched"] = batched_leg(torch, np)
            log(f"[bench] batched: {json.dumps(forms['batched'])}")
        except Exception as e:  # reported, never hides the headline
            forms["batched"] = {"error": repr(e)}
    if args.scf_run:
        log("[bench] Algorithm 3 to convergence ...")
        try:
            out["scf_run"] = scf_run_leg(np, w, args.precision)
            log(f"[bench] scf_run: {json.dumps(out['scf_run'])}")
        except Exception as e:  # reported, never hides the headline
            out["scf_run"] = {"error": repr(e)}
    if args.compare:
        log("[bench] Algorithm 3 against the direct SCF ...")
        try:
            out["compare"] = compare_leg(np)
        except Exception as e:  # reported, never hides the headline
            out["compare"] = {"error": repr(e)}
    if not args.no_differentiation and args.mode == "step":
        log("[bench] differentiation form ...")
        try:
            out["differentiation"] = differentiation_leg(np)
            log(f"[bench] differentiation: {json.dumps(out['differentiation'])}")
        except Exception as e:  # reported, never hides the headline
            out["differentiation"] = {"error": repr(e)}
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle) ...")
        n_inner = int(np.median([r["inner_iters"] for r in reps])) if reps else None
        out["cpu_baseline"] = cpu_baseline(k, tol, n_inner=n_inner, N_full=N)
        if reps:
            out["cpu_baseline"]["step_gpu_over_cpu"] = out["cpu_baseline"]["step_extrapolated_s"] / (ms_per_step * 1e-3)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
