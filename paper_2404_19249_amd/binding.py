"""ctypes binding of the C ABI in include/ks.h.

Argument marshalling only: every computation runs in the HIP library.
PyTorch supplies device memory and the stream.  Loading fails loudly when the
built library is missing; there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libks.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ks.h")

KS_OK, KS_NOT_CONVERGED, KS_WARN_DEGENERATE = 0, 1, 2
STATUS_NAMES = {0: "KS_OK", 1: "KS_NOT_CONVERGED", 2: "KS_WARN_DEGENERATE", -1: "KS_ERR_ARG",
                -2: "KS_ERR_HIP", -3: "KS_ERR_NOMEM", -4: "KS_ERR_MESH", -5: "KS_ERR_BREAKDOWN",
                -6: "KS_ERR_EIG", -7: "KS_ERR_STATE"}
XC = {"none": 0, "x_only": 1, "x_pz81": 2}
HARTREE = {"off": 0, "multipole": 1, "multipole_literal": 2}
PREC = {"fp64": 0, "mixed": 1, "block_cg": 2}


class MeshDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("n_elems", C.c_int32), ("order", C.c_int32),
                ("coords_host", C.POINTER(C.c_double)), ("elems_host", C.POINTER(C.c_int32)),
                ("dirichlet_host", C.POINTER(C.c_uint8)), ("L", C.c_double)]


class MetricParams(C.Structure):
    _fields_ = [("eps", C.c_double), ("h_min", C.c_double), ("h_max", C.c_double)]


class QuadDesc(C.Structure):
    _fields_ = [("n_q", C.c_int32), ("bary_host", C.POINTER(C.c_double)),
                ("w_host", C.POINTER(C.c_double))]


class AtomsDesc(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("Z_host", C.POINTER(C.c_double)),
                ("R_host", C.POINTER(C.c_double))]


class Options(C.Structure):
    _fields_ = [("mu", C.c_double), ("n_H", C.c_int32), ("xc_mode", C.c_int32),
                ("hartree_mode", C.c_int32), ("k_max", C.c_int32), ("tol_solve", C.c_double),
                ("tol_inner", C.c_double), ("tol_poisson", C.c_double),
                ("max_it_solve", C.c_int32), ("max_it_inner", C.c_int32),
                ("max_it_poisson", C.c_int32), ("anderson_depth", C.c_int32),
                ("anderson_beta", C.c_double), ("mixed_inner_tol", C.c_double),
                ("deterministic", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int32 * 64), ("refinements", C.c_int32), ("converged", C.c_int32),
                ("relres", C.c_double * 64), ("seconds", C.c_double)]


class StepReport(C.Structure):
    _fields_ = [("E_total", C.c_double), ("E_band", C.c_double), ("E_H", C.c_double),
                ("E_xc", C.c_double), ("E_vxc", C.c_double), ("E_nn", C.c_double),
                ("res_inner", C.c_double), ("inner_iters", C.c_int32),
                ("poisson_iters", C.c_int32), ("rank", C.c_int32), ("status_solve", C.c_int32),
                ("solve", SolveStats), ("seconds", C.c_double * 8), ("res_outer", C.c_double)]


class RunReport(C.Structure):
    _fields_ = [("steps", C.c_int32), ("converged", C.c_int32), ("inner_iters", C.c_int32),
                ("poisson_iters", C.c_int32), ("res_outer", C.c_double), ("E_total", C.c_double),
                ("E_KS", C.c_double), ("seconds", C.c_double)]


class DirectReport(C.Structure):
    _fields_ = [("scf_iters", C.c_int32), ("eig_iters", C.c_int32), ("poisson_iters", C.c_int32),
                ("converged", C.c_int32), ("res", C.c_double), ("eig_res", C.c_double),
                ("E_total", C.c_double), ("E_band", C.c_double), ("E_H", C.c_double),
                ("E_xc", C.c_double), ("E_vxc", C.c_double), ("E_nn", C.c_double),
                ("seconds", C.c_double)]


class BatchStats(C.Structure):
    _fields_ = [("seconds", C.c_double), ("n", C.c_int32), ("system_seconds", C.c_double * 256),
                ("iters", C.c_int32 * 256), ("relres", C.c_double * 256),
                ("status", C.c_int32 * 256)]


_P = C.c_void_p
_SIGS = {
    "ks_options_default": (C.c_int, [C.POINTER(Options)]),
    "ks_set_options": (C.c_int, [_P, C.POINTER(Options)]),
    "ks_create": (C.c_int, [C.POINTER(MeshDesc), C.POINTER(QuadDesc), C.POINTER(AtomsDesc),
                            C.POINTER(Options), _P, C.POINTER(_P)]),
    "ks_create_nonnested": (C.c_int, [C.POINTER(MeshDesc), C.POINTER(MeshDesc), C.POINTER(QuadDesc),
                                      C.POINTER(AtomsDesc), C.POINTER(Options), _P, C.POINTER(_P)]),
    "ks_destroy": (C.c_int, [_P]),
    "ks_last_error": (C.c_char_p, []),
    "ks_get_sizes": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "ks_assemble": (C.c_int, [_P, _P, C.c_int32, C.POINTER(C.c_double), _P, _P, _P,
                              C.POINTER(C.c_double)]),
    "ks_export_operator": (C.c_int, [_P, C.c_int32, _P, _P, _P]),
    "ks_block_solve": (C.c_int, [_P, _P, C.POINTER(C.c_double), C.c_int32, C.c_int32, _P,
                                 C.POINTER(SolveStats)]),
    "ks_block_solve_rhs": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, C.c_double, _P,
                                     C.POINTER(SolveStats)]),
    "ks_augmented_project": (C.c_int, [_P, _P, C.c_int32, C.c_int32, _P]),
    "ks_small_eig": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, _P, C.POINTER(C.c_double),
                               C.POINTER(C.c_int32)]),
    "ks_small_eig_noalloc": (C.c_int, [_P, _P, C.c_int32, C.c_int32, _P, C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32), _P]),
    "ks_initial_guess": (C.c_int, [_P, C.c_int32, _P, C.POINTER(C.c_double)]),
    "ks_spmm_config": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "ks_time_kernel": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double)]),
    "ks_autotune": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_double)]),
    "ks_autotune_cached": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_char_p, C.POINTER(C.c_int32)]),
    "ks_set_external": (C.c_int, [_P, _P, C.POINTER(C.c_double)]),
    "ks_step_energy": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "ks_step_backward": (C.c_int, [_P, C.c_double, _P, C.POINTER(C.c_double), C.POINTER(SolveStats)]),
    "ks_debug_buffer": (C.c_int, [_P, C.c_char_p, _P, C.c_int64]),
    "ks_batch_create": (C.c_int, [C.c_int32, C.POINTER(_P), C.POINTER(C.c_int32), C.c_int32,
                                  C.POINTER(_P)]),
    "ks_batch_info": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "ks_batch_set_layout": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "ks_batch_block_solve": (C.c_int, [_P, C.POINTER(_P), C.POINTER(C.POINTER(C.c_double)),
                                       C.POINTER(_P), C.POINTER(BatchStats)]),
    "ks_batch_autotune": (C.c_int, [_P, C.POINTER(_P), C.POINTER(C.POINTER(C.c_double)), C.c_int32,
                                    C.POINTER(C.c_double)]),
    "ks_batch_destroy": (C.c_int, [_P]),
    "ks_scf_step": (C.c_int, [_P, _P, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double),
                              C.c_int32, _P, C.POINTER(StepReport)]),
    "ks_mesh_metric": (C.c_int, [C.POINTER(MeshDesc), _P, C.c_int32, C.POINTER(C.c_double),
                                 C.POINTER(MetricParams), _P, _P]),
    "ks_move_nodes": (C.c_int, [C.POINTER(MeshDesc), _P, C.c_double, C.c_int32, C.POINTER(C.c_double),
                                C.POINTER(C.c_int32), _P]),
    "ks_interpolate_field": (C.c_int, [C.POINTER(MeshDesc), _P, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                       _P, _P]),
    "ks_step_backward_truncated": (C.c_int, [_P, C.c_double, C.c_int32, _P, C.POINTER(C.c_double),
                                             C.POINTER(SolveStats)]),
    "ks_step_backward_mesh": (C.c_int, [_P, C.c_double, _P, _P, _P, C.POINTER(C.c_double),
                                        C.POINTER(SolveStats)]),
    "ks_block_solve_vjp": (C.c_int, [_P, _P, _P, C.c_int32, C.c_double, C.c_int32, C.c_int32, _P, _P, _P, _P,
                                     C.POINTER(C.c_int32)]),
    "ks_stream_probe": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double), _P]),
    "ks_interpolate": (C.c_int, [_P, C.POINTER(MeshDesc), _P, C.c_int32, C.c_int32, _P]),
    "ks_direct_scf": (C.c_int, [_P, _P, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double),
                                C.c_double, C.c_int32, C.c_double, C.c_int32, _P, C.POINTER(DirectReport)]),
    "ks_scf_run": (C.c_int, [_P, _P, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double),
                             C.c_int32, C.c_double, C.c_int32, _P, C.POINTER(RunReport)]),
}

_lib = None


def load_library(path=None):
    """Load libks.so (built by paper_2404_19249_amd.build); raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} is missing (run __graft_entry__.build())")
    lib = C.CDLL(p)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


class KSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code, lib=None):
    if code < 0:
        lib = lib or load_library()
        raise KSError(code, lib.ks_last_error().decode(errors="replace"))
    return code


def dptr(x):
    """Host numpy float64 array -> double*."""
    return x.ctypes.data_as(C.POINTER(C.c_double))


def header_functions():
    """Names of the functions declared in include/ks.h."""
    import re
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(ks_\w+)\s*\(", txt, re.M)))
