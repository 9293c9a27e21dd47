"""CPU checks of the C ABI: the library loads, exports every entry point that
include/gbp.h declares, and rejects bad meshes before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import gbp_inputs as gi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gbp.h")
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))
LIB = os.path.join(ROOT, "paper_2308_08410_amd", "libgbp.so")


def declared(headers=None):
    txt = "".join(open(h).read() for h in (headers or HEADERS))
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*(gbp_\w+)\s*\(", txt, re.M)))


def test_header_declares_entry_points():
    names = declared([HEADER])
    for need in ["gbp_plan_create", "gbp_plan_destroy", "gbp_eikonal_forward", "gbp_eikonal_backward",
                 "gbp_parent_map", "gbp_ecg_forward", "gbp_ecg_backward", "gbp_ecg_loss", "gbp_adam_step",
                 "gbp_last_error"]:
        assert need in names


def test_test_hooks_stay_out_of_the_public_header():
    assert "gbp_plan_set_stamp_base" not in declared([HEADER])
    assert "gbp_plan_set_stamp_base" in declared()


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first: python -m paper_2308_08410_amd.build"
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


def test_binding_imports_and_reports_version():
    from paper_2308_08410_amd import binding as B
    assert "gfx950" in B.version()


def _create(xyz, tets):
    from paper_2308_08410_amd import binding as B
    h = ctypes.c_void_p()
    xyz = np.ascontiguousarray(xyz, np.float32)
    tets = np.ascontiguousarray(tets, np.int32)
    rc = B._plan_create(xyz.ctypes.data, len(xyz), tets.ctypes.data, len(tets), None, ctypes.byref(h))
    return rc, B._last_error().decode()


def test_plan_rejects_bad_meshes_before_gpu():
    xyz, tets = gi.kuhn_cube(2)
    bad = tets.copy()
    bad[3, 2] = len(xyz) + 5
    rc, msg = _create(xyz, bad)
    assert rc == -1 and "out of range" in msg
    bad = tets.copy()
    bad[0, 1] = bad[0, 0]
    rc, msg = _create(xyz, bad)
    assert rc == -1 and "repeats" in msg
    flat = xyz.copy()
    flat[:, 2] = 0.0                                # every element collapses
    rc, msg = _create(flat, tets)
    assert rc == -2 and "degenerate" in msg
    nan = xyz.copy()
    nan[4, 0] = np.nan
    rc, msg = _create(nan, tets)
    assert rc == -4
    rc, msg = _create(xyz[:0], tets)
    assert rc == -1


def test_mlp_entry_points_validate_before_gpu():
    lib = ctypes.CDLL(LIB)
    h = ctypes.c_void_p()
    for bad in (0, -3, (1 << 21) + 1):
        assert lib.gbp_mlp_create(bad, ctypes.c_uint64(0), ctypes.byref(h)) == -1
    f = lib.gbp_mlp_features
    f.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 5
    norm = (ctypes.c_float * 5)(0, 0, 0, 1, 1)
    fake = ctypes.c_void_p(16)   # never dereferenced: the checks run first
    # 9 roots, n_rows > n_v without a row list, zero length scale, T without target
    assert f(fake, fake, None, 10, None, 5, fake, fake, 9, norm, None, fake, None, None) == -1
    assert f(fake, fake, None, 10, None, 11, fake, fake, 2, norm, None, fake, None, None) == -1
    norm0 = (ctypes.c_float * 5)(0, 0, 0, 0, 1)
    assert f(fake, fake, None, 10, None, 5, fake, fake, 2, norm0, None, fake, None, None) == -1
    assert f(fake, fake, None, 10, None, 5, fake, fake, 2, norm, fake, fake, None, None) == -1


def test_triangle_plan_rejects_bad_meshes_before_gpu():
    from paper_2308_08410_amd import binding as B
    xy, tris = gi.square_tri(2)

    def create(x, t):
        h = ctypes.c_void_p()
        x = np.ascontiguousarray(x, np.float32)
        t = np.ascontiguousarray(t, np.int32)
        return B._tri_create(x.ctypes.data, len(x), t.ctypes.data, len(t), ctypes.byref(h))

    bad = tris.copy()
    bad[1, 2] = -1
    assert create(xy, bad) == -1
    bad = tris.copy()
    bad[0, 2] = bad[0, 1]
    assert create(xy, bad) == -1
    flat = xy.copy()
    flat[:, 1] = 0.0
    assert create(flat, tris) == -2
    nan = xy.copy()
    nan[3, 0] = np.inf
    assert create(nan, tris) == -4


def test_local_solve_and_lead_field_validate_before_gpu():
    lib = ctypes.CDLL(LIB)
    f = lib.gbp_local_solve
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                  ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    fake = ctypes.c_void_p(16)   # never dereferenced: the checks run first
    assert f(fake, fake, -1, 0, 1, None, 1, fake, None, None, None) == -1        # n < 0
    assert f(fake, fake, 4, 2, 1, None, 1, fake, None, None, None) == -1         # solver
    assert f(fake, fake, 4, 1, 0, None, 1, fake, None, None, None) == -1         # n_f
    assert f(fake, fake, 4, 1, 8, None, 3, fake, None, None, None) == -1         # step-constant mode
    assert f(None, fake, 4, 0, 1, None, 1, fake, None, None, None) == -1         # missing Q
    assert f(fake, fake, 0, 0, 1, None, 1, None, None, None, None) == 0          # empty batch


def test_fista_iterations_validate_before_gpu():
    lib = ctypes.CDLL(LIB)
    f = lib.gbp_fista_iterations
    f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_int, ctypes.c_void_p,
                  ctypes.c_void_p]
    fake = ctypes.c_void_p(16)   # never dereferenced: the checks run first
    assert f(fake, -1, 1e-3, 32, fake, None) == -1               # n < 0
    assert f(fake, 4, -1e-3, 32, fake, None) == -1               # negative tolerance
    assert f(fake, 4, float("nan"), 32, fake, None) == -1        # NaN tolerance
    assert f(fake, 4, float("inf"), 32, fake, None) == -1        # infinite tolerance
    assert f(fake, 4, 1e-3, 0, fake, None) == -1                 # n_max < 1
    assert f(fake, 4, 1e-3, 100001, fake, None) == -1            # n_max too large
    assert f(None, 4, 1e-3, 32, fake, None) == -1                # missing lip
    assert f(fake, 4, 1e-3, 32, None, None) == -1                # missing output
    assert f(None, 0, 0.0, 1, None, None) == 0                   # empty batch
    plan_set = lib.gbp_plan_set_fista_tolerance
    plan_set.argtypes = [ctypes.c_void_p, ctypes.c_float]
    assert plan_set(None, 1e-3) != 0                             # no plan
