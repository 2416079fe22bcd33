"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes as C

import numpy as np
import pytest

import paper_2404_19249_amd as P
from paper_2404_19249_amd import binding as B


def test_library_exports_every_header_function():
    lib = P.load_library()
    names = P.header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(B._SIGS) == set(names)


def test_options_defaults_follow_the_paper():
    lib = P.load_library()
    o = B.Options()
    assert lib.ks_options_default(C.byref(o)) == 0
    assert o.anderson_depth == 5 and abs(o.anderson_beta - 0.7) < 1e-15
    assert o.mu < 0          # selects 8 M sum Z^2
    assert o.tol_solve == 1e-8


def test_create_rejects_bad_arguments_without_gpu():
    lib = P.load_library()
    h = C.c_void_p()
    assert lib.ks_create(None, None, None, None, None, C.byref(h)) == -1
    assert b"null" in lib.ks_last_error()
    coords = np.zeros((4, 3))
    elems = np.array([[0, 1, 2, 3]], dtype=np.int32)
    d = np.zeros(4, np.uint8)
    mesh = B.MeshDesc(4, 1, 3, coords.ctypes.data_as(C.POINTER(C.c_double)),
                      elems.ctypes.data_as(C.POINTER(C.c_int32)),
                      d.ctypes.data_as(C.POINTER(C.c_uint8)), 1.0)
    bary = np.zeros((8, 4)); w = np.zeros(8)
    quad = B.QuadDesc(8, bary.ctypes.data_as(C.POINTER(C.c_double)),
                      w.ctypes.data_as(C.POINTER(C.c_double)))
    atoms = B.AtomsDesc(0, None, None)
    assert lib.ks_create(C.byref(mesh), C.byref(quad), C.byref(atoms), None, None,
                         C.byref(h)) == -1
    assert b"order" in lib.ks_last_error()
    mesh.order = 1
    elems[0, 3] = 7          # node id out of range
    assert lib.ks_create(C.byref(mesh), C.byref(quad), C.byref(atoms), None, None,
                         C.byref(h)) == -4
    quad.n_q = 5
    assert lib.ks_create(C.byref(mesh), C.byref(quad), C.byref(atoms), None, None,
                         C.byref(h)) == -1


def test_null_context_calls_fail_cleanly():
    lib = P.load_library()
    assert lib.ks_block_solve(None, None, None, 1, 0, None, None) == -1
    assert lib.ks_scf_step(None, None, None, 1, None, 0, None, None) == -1
    assert lib.ks_destroy(None) == 0


def test_product_never_imports_the_oracle():
    import pathlib
    pkg = pathlib.Path(P.__file__).parent
    for f in pkg.rglob("*.py"):
        txt = f.read_text()
        assert "import oracle" not in txt and "from oracle" not in txt, f
    for f in pkg.rglob("*.hip"):
        assert "oracle" not in f.read_text().lower(), f
