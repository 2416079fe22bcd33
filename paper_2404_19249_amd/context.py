"""Python front end of the library: one KSContext per mesh.

Every method marshals torch tensors (device memory) and numpy arrays (host
inputs) into one C ABI call; the arithmetic happens in the HIP kernels.
"""
import ctypes as C
import os

import numpy as np

from . import binding as B


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class KSContext:
    """Per-mesh state of the augmented subspace step on one GPU."""

    def __init__(self, coords, elems, dirichlet, order, L, quad_bary, quad_w, Z, R, *, n_H=4,
                 mu=None, xc="x_pz81", hartree="multipole", k_max=8, tol_solve=1e-8,
                 tol_inner=1e-8, tol_poisson=1e-10, max_it_solve=5000, max_it_inner=50,
                 max_it_poisson=20000, anderson_depth=5, anderson_beta=0.7,
                 mixed_inner_tol=1e-5, device=0, stream=None, coarse=None):
        """coarse: optional nonnested coarse P1 mesh (an object with coords,
        elems, dirichlet, L), giving S_H on that mesh (ks_create_nonnested)
        instead of the uniform n_H mesh."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("KSContext needs a ROCm GPU; none is visible")
        self.torch = torch
        self.lib = B.load_library()
        self.device = torch.device("cuda", device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        # host inputs are copied by ks_create; keep them alive for the call
        self._coords = _f64(coords)
        self._elems = _i32(elems)
        self._dir = np.ascontiguousarray(dirichlet, dtype=np.uint8)
        self._bary = _f64(quad_bary)
        self._w = _f64(quad_w)
        self._Z = _f64(Z)
        self._R = _f64(np.asarray(R).reshape(-1, 3))
        mesh = B.MeshDesc(self._coords.shape[0], self._elems.shape[0], int(order),
                          self._coords.ctypes.data_as(C.POINTER(C.c_double)),
                          self._elems.ctypes.data_as(C.POINTER(C.c_int32)),
                          self._dir.ctypes.data_as(C.POINTER(C.c_uint8)), float(L))
        quad = B.QuadDesc(self._w.shape[0], self._bary.ctypes.data_as(C.POINTER(C.c_double)),
                          self._w.ctypes.data_as(C.POINTER(C.c_double)))
        atoms = B.AtomsDesc(self._Z.shape[0], self._Z.ctypes.data_as(C.POINTER(C.c_double)),
                            self._R.ctypes.data_as(C.POINTER(C.c_double)))
        opt = B.Options()
        B.check(self.lib.ks_options_default(C.byref(opt)))
        opt.mu = -1.0 if mu is None else float(mu)
        opt.n_H = int(n_H)
        opt.xc_mode = B.XC[xc]
        opt.hartree_mode = B.HARTREE[hartree]
        opt.k_max = int(k_max)
        opt.tol_solve, opt.tol_inner, opt.tol_poisson = tol_solve, tol_inner, tol_poisson
        opt.max_it_solve, opt.max_it_inner, opt.max_it_poisson = max_it_solve, max_it_inner, max_it_poisson
        opt.anderson_depth, opt.anderson_beta = anderson_depth, anderson_beta
        opt.mixed_inner_tol = mixed_inner_tol
        self.opt = opt
        h = C.c_void_p()
        cmesh = None
        if coarse is not None:
            self._c_coords = _f64(coarse.coords)
            self._c_elems = _i32(coarse.elems)
            self._c_dir = np.ascontiguousarray(coarse.dirichlet, dtype=np.uint8)
            cmesh = B.MeshDesc(self._c_coords.shape[0], self._c_elems.shape[0], 1,
                               self._c_coords.ctypes.data_as(C.POINTER(C.c_double)),
                               self._c_elems.ctypes.data_as(C.POINTER(C.c_int32)),
                               self._c_dir.ctypes.data_as(C.POINTER(C.c_uint8)), float(coarse.L))
        with torch.cuda.device(self.device):
            B.check(self.lib.ks_create_nonnested(C.byref(mesh), C.byref(cmesh) if cmesh is not None else None,
                                                 C.byref(quad), C.byref(atoms), C.byref(opt),
                                                 C.c_void_p(self.stream.cuda_stream), C.byref(h)), self.lib)
        self.h = h
        sz = (C.c_double * 11)()
        B.check(self.lib.ks_get_sizes(self.h, sz))
        self.N, self.n_nodes, self.n_elems, self.n_q, self.N_H, self.nnz, self.n_loc, \
            self.n_colours, self.ld_z = [int(v) for v in sz[:9]]
        self.mu = float(sz[9])
        self.mg_levels = int(sz[10])
        self.k_max = k_max

    _SETTABLE = ("tol_solve", "tol_inner", "tol_poisson", "max_it_solve", "max_it_inner",
                 "max_it_poisson", "anderson_depth", "anderson_beta", "mixed_inner_tol")

    def set_options(self, **kw):
        """Change tolerances, iteration limits or Anderson parameters of the
        live context (ks_set_options); other options are fixed at creation."""
        opt = B.Options()
        C.memmove(C.byref(opt), C.byref(self.opt), C.sizeof(B.Options))
        for key, v in kw.items():
            if key not in self._SETTABLE:
                raise KeyError(f"option {key} cannot change after creation")
            setattr(opt, key, v)
        B.check(self.lib.ks_set_options(self.h, C.byref(opt)), self.lib)
        self.opt = opt

    @classmethod
    def from_workload(cls, w, **kw):
        kw.setdefault("n_H", w.n_H)
        kw.setdefault("xc", "x_pz81" if w.xc else "none")
        kw.setdefault("hartree", "multipole" if w.hartree else "off")
        kw.setdefault("k_max", max(w.k, 1))
        m = w.mesh
        return cls(m.coords, m.elems, m.dirichlet, m.order, m.L, w.quad.bary, w.quad.w,
                   w.atoms.Z, w.atoms.R, **kw)

    def close(self):
        if getattr(self, "h", None):
            self.lib.ks_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- helpers
    def empty(self, *shape, dtype=None):
        return self.torch.empty(*shape, dtype=dtype or self.torch.float64, device=self.device)

    def _ptr(self, t):
        if t is None:
            return None
        assert t.is_contiguous() and t.device == self.device, "device tensor expected"
        return C.c_void_p(t.data_ptr())

    # ------------------------------------------------------------------- API
    def assemble(self, psi=None, occ=None, want_fields=True):
        """ks_assemble: S of the density of psi; returns rho_q, veff_q, V_H
        (nodes) and the energy terms."""
        k = 0 if psi is None else psi.shape[1]
        occ_a = None if psi is None else _f64(occ)
        out = {}
        if want_fields:
            out["rho_q"] = self.empty(self.n_elems, self.n_q)
            out["veff_q"] = self.empty(self.n_elems, self.n_q)
            out["vh_nodes"] = self.empty(self.n_nodes)
        e = np.zeros(5)
        B.check(self.lib.ks_assemble(self.h, self._ptr(psi), k,
                                     None if occ_a is None else B.dptr(occ_a),
                                     self._ptr(out.get("rho_q")), self._ptr(out.get("veff_q")),
                                     self._ptr(out.get("vh_nodes")), B.dptr(e)), self.lib)
        out["energies"] = {"E_H": e[0], "E_xc": e[1], "E_vxc": e[2], "E_ext": e[3],
                           "poisson_iters": int(e[4])}
        return out

    def export_operator(self, which):
        """CSR arrays (host numpy) of operator `which` (0 S, 1 K, 2 M, 3 A^L, 4 M[V_nl])."""
        rp = self.empty(self.N + 1, dtype=self.torch.int32)
        cl = self.empty(self.nnz, dtype=self.torch.int32)
        vl = self.empty(self.nnz)
        B.check(self.lib.ks_export_operator(self.h, int(which), self._ptr(rp), self._ptr(cl),
                                            self._ptr(vl)), self.lib)
        return rp.cpu().numpy(), cl.cpu().numpy(), vl.cpu().numpy()

    @staticmethod
    def _stats(st, k):
        return {"iters": list(st.iters[:k]), "relres": list(st.relres[:k]),
                "refinements": st.refinements, "converged": bool(st.converged),
                "seconds": st.seconds}

    def block_solve(self, psi_old, lam, precision="fp64", out=None):
        k = psi_old.shape[1]
        lam_a = _f64(lam)
        out = out if out is not None else self.empty(self.N, k)
        st = B.SolveStats()
        code = B.check(self.lib.ks_block_solve(self.h, self._ptr(psi_old), B.dptr(lam_a), k,
                                               B.PREC[precision], self._ptr(out), C.byref(st)),
                       self.lib)
        s = self._stats(st, k)
        s["status"] = code
        return out, s

    def block_solve_rhs(self, Bm, X0=None, precision="fp64", tol=0.0):
        k = Bm.shape[1]
        X = self.empty(self.N, k)
        st = B.SolveStats()
        code = B.check(self.lib.ks_block_solve_rhs(self.h, self._ptr(Bm), self._ptr(X0), k,
                                                   B.PREC[precision], float(tol), self._ptr(X),
                                                   C.byref(st)), self.lib)
        s = self._stats(st, k)
        s["status"] = code
        return X, s

    def block_solve_vjp(self, Bm, Xbar, X0=None, tol=1e-10, max_it=500, seg=8):
        """ks_block_solve_vjp: the truncated FP64 solve X of S X = Bm and, for
        L = sum(Xbar * X), dL/dV at the quadrature points and dL/dBm."""
        k = Bm.shape[1]
        X = self.empty(self.N, k)
        g = self.empty(self.n_elems, self.n_q)
        Bbar = self.empty(self.N, k)
        its = (C.c_int32 * k)()
        B.check(self.lib.ks_block_solve_vjp(self.h, self._ptr(Bm.contiguous()),
                                            self._ptr(None if X0 is None else X0.contiguous()), k, float(tol),
                                            int(max_it), int(seg), self._ptr(Xbar.contiguous()), self._ptr(X),
                                            self._ptr(g), self._ptr(Bbar), its), self.lib)
        return X, g, Bbar, list(its)

    def augmented_project(self, psi_hat, which):
        k = psi_hat.shape[1]
        m = self.N_H + k
        F = self.empty(m, m)
        B.check(self.lib.ks_augmented_project(self.h, self._ptr(psi_hat), k, int(which),
                                              self._ptr(F)), self.lib)
        return F

    def small_eig(self, FA, FB, k):
        m = FA.shape[0]
        U = self.empty(m, k)
        lam = np.zeros(k)
        rank = C.c_int32()
        B.check(self.lib.ks_small_eig(self.h, self._ptr(FA.contiguous()), self._ptr(FB.contiguous()),
                                      m, k, self._ptr(U), B.dptr(lam), C.byref(rank)), self.lib)
        return U, lam, rank.value

    def time_kernel(self, which, k, reps=20):
        """Mean launch duration (ms) of a block-PCG phase; see ks_time_kernel."""
        ms = C.c_double()
        B.check(self.lib.ks_time_kernel(self.h, int(which), int(k), int(reps), C.byref(ms)), self.lib)
        return ms.value

    def set_external(self, vext_q=None, R=None):
        """ks_set_external: new V_ext at the quadrature points or new nuclei."""
        if R is not None:
            self._R = _f64(np.asarray(R).reshape(-1, 3))
            B.check(self.lib.ks_set_external(self.h, None, B.dptr(self._R)), self.lib)
        else:
            B.check(self.lib.ks_set_external(self.h, self._ptr(vext_q.contiguous()), None), self.lib)

    def step_energy(self):
        """ks_step_energy of the last scf_step."""
        e = np.zeros(6)
        B.check(self.lib.ks_step_energy(self.h, B.dptr(e)), self.lib)
        return dict(zip(["KS", "kin", "ext", "H_step", "xc", "nn"], e))

    def step_backward(self, dE=1.0, want_forces=True, truncated=False, seg=8):
        """ks_step_backward (implicit adjoint of the BVPs) or, with truncated,
        ks_step_backward_truncated (reverse mode through the truncated FP64
        PCG): (g_q device tensor, forces [n_atoms][3] numpy, stats)."""
        g = self.empty(self.n_elems, self.n_q)
        F = np.zeros((len(self._Z), 3)) if want_forces else None
        st = B.SolveStats()
        Fp = None if F is None else B.dptr(F)
        if truncated:
            B.check(self.lib.ks_step_backward_truncated(self.h, float(dE), int(seg), self._ptr(g), Fp,
                                                        C.byref(st)), self.lib)
        else:
            B.check(self.lib.ks_step_backward(self.h, float(dE), self._ptr(g), Fp, C.byref(st)), self.lib)
        return g, F, self._stats(st, 64)

    def step_backward_mesh(self, dE=1.0, motion=None):
        """ks_step_backward_mesh: (dE/dX device [n_nodes][3], g_q device
        tensor, forces [n_atoms][3] numpy, stats).  With motion (device
        [n_nodes][n_atoms]: node n moves by motion[n][a] dR_a) the forces
        carry the mesh-motion terms; without it they are the fixed-mesh
        forces."""
        dX = self.empty(self.n_nodes, 3)
        g = self.empty(self.n_elems, self.n_q)
        F = np.zeros((len(self._Z), 3))
        st = B.SolveStats()
        if motion is not None:
            import torch
            if motion.dtype != torch.float64 or tuple(motion.shape) != (self.n_nodes, len(self._Z)):
                raise ValueError(f"motion must be float64 [n_nodes][n_atoms] = [{self.n_nodes}][{len(self._Z)}]")
        mp = None if motion is None else self._ptr(motion.contiguous())
        B.check(self.lib.ks_step_backward_mesh(self.h, float(dE), mp, self._ptr(dX), self._ptr(g), B.dptr(F),
                                               C.byref(st)), self.lib)
        return dX, g, F, self._stats(st, 64)

    def spmm_config(self):
        """ks_spmm_config: the SpMM-phase kernel of each solver."""
        o = (C.c_int32 * 9)()
        B.check(self.lib.ks_spmm_config(self.h, o), self.lib)
        return {"ng_fp64": o[0], "ng_fp32": o[1], "ng_poisson": o[2], "tile_fp64": o[3],
                "tile_fp32": o[4], "tile_poisson": o[5], "tile_threads_fp64": o[6],
                "tile_threads_fp32": o[7], "tile_threads_poisson": o[8]}

    def autotune(self, k, reps=10):
        """ks_autotune: pick the SpMM phase kernel (row kernel lanes-per-row
        split, or halo-tile row-block size and workgroup size) per solver."""
        rep = (C.c_double * 75)()
        B.check(self.lib.ks_autotune(self.h, int(k), int(reps), rep), self.lib)
        r = list(rep)
        names = ["fp64", "fp32", "poisson"]
        out = {}
        for w, n in enumerate(names):
            out[f"ng_{n}"] = int(r[w])
            out[f"tile_{n}"] = int(r[3 + w])
            out[f"tile_threads_{n}"] = int(r[6 + w])
            out[f"row_ms_{n}"] = dict(zip([1, 2, 4, 8], r[9 + 4 * w: 13 + 4 * w]))
            t = r[21 + 18 * w: 39 + 18 * w]
            out[f"tile_ms_{n}"] = {f"{br}x{tb}": t[3 * i + j]
                                   for i, br in enumerate([32, 64, 85, 128, 170, 256])
                                   for j, tb in enumerate([256, 512, 1024])}
        return out

    def autotune_cached(self, k, path, reps=10):
        """ks_autotune_cached: apply the cached SpMM-phase choice for this
        device, order, size class, nonzeros per row and k from the text file
        at `path`, or tune and append it.  Returns True on a cache hit."""
        hit = C.c_int32(0)
        B.check(self.lib.ks_autotune_cached(self.h, int(k), int(reps), os.fsencode(path), C.byref(hit)),
                self.lib)
        return bool(hit.value)

    def debug_buffer(self, name, n):
        """Copy of an internal buffer (diagnostics)."""
        t = self.empty(n)
        B.check(self.lib.ks_debug_buffer(self.h, name.encode(), self._ptr(t), int(n)), self.lib)
        return t

    def initial_guess(self, k):
        psi = self.empty(self.N, k)
        lam = np.zeros(k)
        B.check(self.lib.ks_initial_guess(self.h, k, self._ptr(psi), B.dptr(lam)), self.lib)
        return psi, lam

    def scf_step(self, psi, lam, occ, precision="fp64", rho_out=None):
        """One iteration of Algorithm 3 in place: psi (device [N][k]) and the
        returned eigenvalues are the new iterate."""
        k = psi.shape[1]
        lam_a = _f64(lam).copy()
        occ_a = _f64(occ)
        rep = B.StepReport()
        code = B.check(self.lib.ks_scf_step(self.h, self._ptr(psi), B.dptr(lam_a), k,
                                            B.dptr(occ_a), B.PREC[precision], self._ptr(rho_out),
                                            C.byref(rep)), self.lib)
        r = {f: getattr(rep, f) for f in ("E_total", "E_band", "E_H", "E_xc", "E_vxc", "E_nn",
                                          "res_inner", "inner_iters", "poisson_iters", "rank",
                                          "status_solve", "res_outer")}
        r["solve"] = self._stats(rep.solve, k)
        r["seconds"] = list(rep.seconds[:6])
        r["status"] = code
        return lam_a, r

    def scf_run(self, psi, lam, occ, tol, max_steps=100, precision="fp64", rho_out=None):
        """Algorithm 3 to convergence (ks_scf_run): steps in place on psi until
        the density changes by less than tol (quadrature L2 norm)."""
        k = psi.shape[1]
        lam_a = _f64(lam).copy()
        occ_a = _f64(occ)
        rep = B.RunReport()
        code = B.check(self.lib.ks_scf_run(self.h, self._ptr(psi), B.dptr(lam_a), k, B.dptr(occ_a),
                                           B.PREC[precision], float(tol), int(max_steps),
                                           self._ptr(rho_out), C.byref(rep)), self.lib)
        r = {f: getattr(rep, f) for f in ("steps", "converged", "inner_iters", "poisson_iters",
                                          "res_outer", "E_total", "E_KS", "seconds")}
        r["status"] = code
        return lam_a, r


    def interpolate(self, src_mesh, psi_src, orthonormalize=False):
        """ks_interpolate: orbitals P1 on src_mesh (coords, elems, dirichlet,
        order 1) carried to this context's interior nodes by Algorithm 1,
        optionally made M-orthonormal there (Cholesky, column order)."""
        k = psi_src.shape[1]
        co, el, di = _f64(src_mesh.coords), _i32(src_mesh.elems), np.ascontiguousarray(src_mesh.dirichlet, np.uint8)
        md = B.MeshDesc(co.shape[0], el.shape[0], int(getattr(src_mesh, "order", 1)),
                        co.ctypes.data_as(C.POINTER(C.c_double)), el.ctypes.data_as(C.POINTER(C.c_int32)),
                        di.ctypes.data_as(C.POINTER(C.c_uint8)), float(getattr(src_mesh, "L", 0.0)))
        out = self.empty(self.N, k)
        B.check(self.lib.ks_interpolate(self.h, C.byref(md), self._ptr(psi_src.contiguous()), k,
                                        int(bool(orthonormalize)), self._ptr(out)), self.lib)
        return out

    def direct_scf(self, psi, lam, occ, tol=1e-8, max_scf=200, tol_eig=1e-9, max_eig=500, rho_out=None):
        """The direct SCF on the fine space (ks_direct_scf), in place on psi:
        LOBPCG eigensolves and Anderson-mixed densities until the density
        changes by less than tol."""
        k = psi.shape[1]
        lam_a = _f64(lam).copy()
        occ_a = _f64(occ)
        rep = B.DirectReport()
        code = B.check(self.lib.ks_direct_scf(self.h, self._ptr(psi), B.dptr(lam_a), k, B.dptr(occ_a),
                                              float(tol), int(max_scf), float(tol_eig), int(max_eig),
                                              self._ptr(rho_out), C.byref(rep)), self.lib)
        r = {f: getattr(rep, f) for f, _ in B.DirectReport._fields_}
        r["status"] = code
        return lam_a, r


class KSBatch:
    """Many independent systems (each a KSContext with an assembled operator)
    solved together: one persistent launch, captured once in a hipGraph and
    replayed by every solve.  The contexts must outlive the batch."""

    def __init__(self, contexts, ks, grid=0):
        self.ctxs = list(contexts)
        self.ks = [int(k) for k in ks]
        self.lib = self.ctxs[0].lib
        self.torch = self.ctxs[0].torch
        n = len(self.ctxs)
        hs = (C.c_void_p * n)(*[c.h for c in self.ctxs])
        karr = (C.c_int32 * n)(*self.ks)
        h = C.c_void_p()
        B.check(self.lib.ks_batch_create(n, hs, karr, int(grid), C.byref(h)), self.lib)
        self.h = h
        self._info()

    def close(self):
        if getattr(self, "h", None):
            self.lib.ks_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _info(self):
        n = len(self.ctxs)
        g = C.c_int32()
        team = (C.c_int32 * n)()
        ng = (C.c_int32 * n)()
        tile = (C.c_int32 * n)()
        B.check(self.lib.ks_batch_info(self.h, C.byref(g), team, ng, tile), self.lib)
        self.grid, self.team, self.ng, self.tile = g.value, list(team), list(ng), list(tile)

    def _args(self, psis, lams):
        n = len(self.ctxs)
        assert len(psis) == n and len(lams) == n
        lam_a = [_f64(l) for l in lams]
        for c, p, l, k in zip(self.ctxs, psis, lam_a, self.ks):
            assert tuple(p.shape) == (c.N, k) and l.size >= k
        pp = (C.c_void_p * n)(*[c._ptr(p).value for c, p in zip(self.ctxs, psis)])
        ll = (C.POINTER(C.c_double) * n)(*[B.dptr(l) for l in lam_a])
        return pp, ll, lam_a

    def set_layout(self, ng=None, tile=None):
        """ks_batch_set_layout: lanes per row and halo-tile row block (0: row
        products) per system; None keeps the current choice."""
        n = len(self.ctxs)
        arr = lambda v: None if v is None else (C.c_int32 * n)(*[int(x) for x in v])
        B.check(self.lib.ks_batch_set_layout(self.h, arr(ng), arr(tile)), self.lib)
        self._info()

    def autotune(self, psis, lams, rounds=3):
        """ks_batch_autotune on these inputs; returns the best launch time (ms)."""
        pp, ll, keep = self._args(psis, lams)
        ms = C.c_double()
        B.check(self.lib.ks_batch_autotune(self.h, pp, ll, int(rounds), C.byref(ms)), self.lib)
        self._info()
        return ms.value

    def block_solve(self, psis, lams, outs=None):
        """psi_hat_s = S_s^{-1} M_s psi_s diag(lam_s + mu_s) for every system s."""
        n = len(self.ctxs)
        pp, ll, keep = self._args(psis, lams)
        outs = outs if outs is not None else [c.empty(c.N, k) for c, k in zip(self.ctxs, self.ks)]
        for c, o, k in zip(self.ctxs, outs, self.ks):
            assert tuple(o.shape) == (c.N, k)
        oo = (C.c_void_p * n)(*[c._ptr(o).value for c, o in zip(self.ctxs, outs)])
        st = B.BatchStats()
        code = B.check(self.lib.ks_batch_block_solve(self.h, pp, ll, oo, C.byref(st)), self.lib)
        return outs, {"status": code, "seconds": st.seconds,
                      "system_seconds": list(st.system_seconds[:n]), "iters": list(st.iters[:n]),
                      "relres": list(st.relres[:n]), "sys_status": list(st.status[:n])}


def stream_probe(kind="copy", nbytes=1 << 30, nontemporal=False, reps=10, stream=None):
    """ks_stream_probe: GB/s of a plain coalesced stream over nbytes-byte
    buffers (kind "read", "copy" or "triad"; read + write bytes counted)."""
    import torch
    lib = B.load_library()
    st = stream or torch.cuda.current_stream()
    out = C.c_double(0.0)
    B.check(lib.ks_stream_probe(int(nbytes), {"read": 0, "copy": 1, "triad": 2}[kind], int(bool(nontemporal)),
                                int(reps), C.byref(out), C.c_void_p(st.cuda_stream)), lib)
    return out.value


class _HostMesh:
    """Host arrays of a P1 mesh kept alive for one call, and its descriptor."""

    def __init__(self, mesh):
        self.co = _f64(mesh.coords)
        self.el = _i32(mesh.elems)
        self.di = np.ascontiguousarray(mesh.dirichlet, np.uint8)
        self.desc = B.MeshDesc(self.co.shape[0], self.el.shape[0], int(getattr(mesh, "order", 1)),
                               self.co.ctypes.data_as(C.POINTER(C.c_double)),
                               self.el.ctypes.data_as(C.POINTER(C.c_int32)),
                               self.di.ctypes.data_as(C.POINTER(C.c_uint8)), float(getattr(mesh, "L", 0.0)))


def _stream(stream):
    import torch
    return C.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


def mesh_metric(mesh, psi, occ, eps, h_min, h_max, stream=None):
    """ks_mesh_metric: the metric of sqrt(rho) (eqs. m1-m2) at every node of
    a P1 mesh; psi device [N][k] (non-Dirichlet nodes ascending).  Returns a
    device tensor [n_nodes][6] (xx, yy, zz, xy, xz, yz)."""
    import torch
    lib = B.load_library()
    hm = _HostMesh(mesh)
    occ_a = _f64(occ)
    out = torch.empty(hm.co.shape[0], 6, dtype=torch.float64, device=psi.device)
    prm = B.MetricParams(float(eps), float(h_min), float(h_max))
    B.check(lib.ks_mesh_metric(C.byref(hm.desc), C.c_void_p(psi.contiguous().data_ptr()), int(psi.shape[1]),
                               B.dptr(occ_a), C.byref(prm), C.c_void_p(out.data_ptr()), _stream(stream)), lib)
    return out


def move_nodes(mesh, metric, omega=0.5, sweeps=1, stream=None):
    """ks_move_nodes: the mesh's nodes after `sweeps` damped metric spring
    sweeps (host [n_nodes][3]) and the number of step halvings."""
    lib = B.load_library()
    hm = _HostMesh(mesh)
    out = np.empty((hm.co.shape[0], 3))
    hv = C.c_int32(0)
    B.check(lib.ks_move_nodes(C.byref(hm.desc), C.c_void_p(metric.contiguous().data_ptr()), float(omega),
                              int(sweeps), B.dptr(out), C.byref(hv), _stream(stream)), lib)
    return out, hv.value


def interpolate_field(src_mesh, field, pts, stream=None):
    """ks_interpolate_field: a P1 nodal field on src_mesh (device [n_nodes][m])
    at the points pts (host [n][3]); returns a device tensor [n][m]."""
    import torch
    lib = B.load_library()
    hm = _HostMesh(src_mesh)
    P = _f64(pts)
    f = field.contiguous()
    m = 1 if f.dim() == 1 else int(f.shape[1])
    out = torch.empty(P.shape[0], m, dtype=torch.float64, device=f.device)
    B.check(lib.ks_interpolate_field(C.byref(hm.desc), C.c_void_p(f.data_ptr()), m, int(P.shape[0]), B.dptr(P),
                                     C.c_void_p(out.data_ptr()), _stream(stream)), lib)
    return out
