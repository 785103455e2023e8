"""The C-ABI library without a GPU: it loads, exports every function the
header declares, validates arguments before any device work, and its host-side
exports agree with the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2001_01655_amd as tm
from paper_2001_01655_amd import _lib as L
from oracle import fem, mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "topomg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tm_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert len(names) >= 25
    lib = C.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert L.LIB.tm_status_string(code).decode() not in ("", "unknown status")


def _setup_status(nel=(8, 4), nu=0.3, Emin=1e-9, E0=1.0, dofs=(0, 1), **opts):
    mesh = L.make_mesh(nel)
    mat = L.make_material(3.0, E0, Emin, nu)
    o = L.default_options(**opts)
    arr = np.asarray(dofs, dtype=np.int64)
    bcs = L.tm_bcs(len(arr), arr.ctypes.data_as(C.POINTER(C.c_int64)))
    h = C.c_void_p()
    # a non-null stand-in for the density buffer: argument checks fail before it is read
    st = L.LIB.tm_setup(C.byref(mesh), C.byref(mat), C.c_void_p(16), C.byref(bcs), C.byref(o), None, None,
                        C.byref(h))
    return st, L.LIB.tm_last_error().decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(nel=(8, 2), n_levels=3), "too many geometric levels"),
    (dict(n_levels=1), "at least two levels"),
    (dict(nu=0.5), "nu"),
    (dict(Emin=2.0), "Emin"),
    (dict(dofs=(0, 10 ** 9)), "out of range"),
    (dict(omega=2.5), "omega"),
    (dict(vcycle_fp=16), "vcycle_fp"),
    (dict(smoother=3), "smoother"),
    (dict(smoother=2, cheb_lower=0.0), "cheb_lower"),
    (dict(n_geometric=1), "n_geometric"),
    (dict(nu_pre=0), "nu_pre"),
    (dict(fine_mfma=2), "fine_mfma"),
    (dict(adapt_iters=-1), "adapt_iters"),
    (dict(cheb_warm_steps=-1), "cheb_warm_steps"),
    (dict(cheb_warm_steps=13), "cheb_warm_steps"),
    (dict(stencil_kernel=4), "stencil_kernel"),
    (dict(sa_lds=2), "sa_lds"),
    (dict(fine_tensor=-1), "fine_tensor"),
])
def test_setup_rejects_bad_arguments_before_device_work(kw, msg):
    st, err = _setup_status(**kw)
    assert st == L.TM_ERR_ARG
    assert msg in err


def test_setup_rejects_an_allocator_without_both_callbacks():
    mesh = L.make_mesh((8, 4))
    mat = L.make_material()
    o = L.default_options()
    arr = np.asarray((0, 1), dtype=np.int64)
    bcs = L.tm_bcs(2, arr.ctypes.data_as(C.POINTER(C.c_int64)))
    h = C.c_void_p()
    half = L.tm_allocator(L.TORCH_ALLOCATOR.alloc, L.FREE_FN(), None)
    st = L.LIB.tm_setup(C.byref(mesh), C.byref(mat), C.c_void_p(16), C.byref(bcs), C.byref(o), C.byref(half),
                        None, C.byref(h))
    assert st == L.TM_ERR_ARG and "allocator" in L.LIB.tm_last_error().decode()
    assert not h.value


def test_plan_bytes_counts_chebyshev_directions():
    """Chebyshev smoothing keeps a direction vector per level and right-hand
    side: the per-RHS increment of the plan grows by at least the fine level's
    FP32 direction."""
    mesh = L.make_mesh((32, 16, 16))
    plan = {(sm, k): L.tm_plan_bytes(mesh, L.default_options(n_levels=3, smoother=sm), k)
            for sm in (0, 2) for k in (1, 4)}
    per_rhs_jac = (plan[0, 4] - plan[0, 1]) / 3
    per_rhs_cheb = (plan[2, 4] - plan[2, 1]) / 3
    assert per_rhs_cheb - per_rhs_jac >= 4 * 3 * 33 * 17 * 17


def test_null_arguments():
    h = C.c_void_p()
    assert L.LIB.tm_setup(None, None, None, None, None, None, None, C.byref(h)) == L.TM_ERR_ARG
    assert L.LIB.tm_solve(None, 1, None, 1e-8, 0, None, None, None, None, None) == L.TM_ERR_ARG
    assert L.LIB.tm_solve_end(None, None, None, None) == L.TM_ERR_STATE
    assert L.LIB.tm_num_levels(None) == 0
    assert L.LIB.tm_stress_stiffness(None, None, 0.1, None) == L.TM_ERR_ARG
    assert L.LIB.tm_apply_stress_stiffness(None, None, None, None) == L.TM_ERR_ARG
    o = L.default_eig_options()
    assert L.LIB.tm_eigs(None, C.byref(o), 1, None, None, None, None, None, None) == L.TM_ERR_ARG


def test_eig_defaults_follow_the_paper():
    o = L.default_eig_options()
    assert (o.nev, o.j_min, o.j_max) == (6, 10, 25)
    assert o.tol == 1e-6 and o.stag_tol == 1e-13 and o.precond_fp == 32


def test_plan_bytes():
    m = L.make_mesh((64, 32, 32))
    o = L.default_options(n_levels=4)
    b1 = tm.tm_plan_bytes(m, o, 1)
    b4 = tm.tm_plan_bytes(m, o, 4)
    assert 0 < b1 < b4
    assert tm.tm_plan_bytes(L.make_mesh((63, 32, 32)), o, 1) > 0      # odd counts coarsen to ceil(n/2)
    with pytest.raises(tm.TmError):
        tm.tm_plan_bytes(L.make_mesh((64, 32, 4)), o, 1)               # 4 -> 2 -> 1 -> (none)


@pytest.mark.parametrize("nel", [(5, 3), (3, 4, 2)])
def test_connectivity_export_matches_oracle(nel):
    conn = tm.tm_export_connectivity(L.make_mesh(nel))
    assert np.array_equal(conn, fem.connectivity(nel))


def test_import_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        L._load()


@pytest.mark.parametrize("radius,transpose,same,msg", [
    (0.0, 0, False, "radius"), (4.5, 0, False, "radius"), (1.5, 2, False, "transpose"), (1.5, 0, True, "overlap"),
])
def test_density_filter_rejects_bad_arguments_before_device_work(radius, transpose, same, msg):
    mesh = L.make_mesh((8, 4))
    a, b = C.c_void_p(0x1000), C.c_void_p(0x1000 if same else 0x2000)
    st = L.LIB.tm_density_filter(C.byref(mesh), radius, transpose, a, b, None)
    assert st == L.TM_ERR_ARG
    assert msg in L.LIB.tm_last_error().decode()
    assert L.LIB.tm_density_filter(C.byref(mesh), 1.5, 0, None, b, None) == L.TM_ERR_ARG


def test_plan_refuses_meshes_past_the_buffer_range():
    """Operator kernels address the fine vectors and the first coarse level's
    stencil through buffer descriptors (range below 2 GiB): a 3D mesh whose
    level-1 FP64 stencil (123 values per node) reaches 2 GiB is refused by both
    admission and setup; the largest that fits is accepted."""
    o = L.default_options(n_levels=6)
    ok = L.make_mesh((256, 256, 256))          # level 1: 129^3 nodes * 984 B = 2.11e9 B
    assert tm.tm_plan_bytes(ok, o, 1) > 0
    big = L.make_mesh((264, 264, 264))         # level 1: 133^3 nodes * 984 B = 2.31e9 B
    with pytest.raises(tm.TmError) as e:
        tm.tm_plan_bytes(big, o, 1)
    assert e.value.status == L.TM_ERR_ARG and "2 GiB" in str(e.value)
    st, err = _setup_status(nel=(264, 264, 264), n_levels=6)
    assert st == L.TM_ERR_ARG and "2 GiB" in err
    # a 2D fine grid whose FP64 vector reaches 2 GiB (dofs of 8 B >= 2^31 B)
    with pytest.raises(tm.TmError):
        tm.tm_plan_bytes(L.make_mesh((11600, 11600)), L.default_options(n_levels=2), 1)
