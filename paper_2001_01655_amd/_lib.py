"""ctypes binding of libtopomg (include/topomg.h): argument marshalling only.

Every function keeps its C name.  Device buffers are torch tensors on the
current HIP device; streams are torch streams.  All computation happens in the
HIP library; if the shared object is missing this module raises at import.
"""
from __future__ import annotations

import ctypes as C
import os

# torch first: its bundled HIP runtime must be the one in the process before
# the library is loaded, so that both resolve to a single runtime (loading the
# library first would bring in a second copy from the system ROCm, and device
# memory allocated by one would be unknown to the other)
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtopomg.so")

TM_OK, TM_NOT_CONVERGED = 0, 1
TM_ERR_ARG, TM_ERR_OOM, TM_ERR_DEVICE, TM_ERR_NOT_SPD, TM_ERR_BREAKDOWN, TM_ERR_STATE = -1, -2, -3, -4, -5, -6
TM_SMOOTH_BLOCK_JACOBI, TM_SMOOTH_POINT_JACOBI, TM_SMOOTH_CHEBYSHEV = 0, 1, 2
TM_OUTER_FCG, TM_OUTER_PCG = 0, 1
TM_LEVEL_FINE, TM_LEVEL_GEOMETRIC, TM_LEVEL_AGGREGATION = 0, 1, 2


class tm_mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nel", C.c_int32 * 3), ("h", C.c_double)]


class tm_material(C.Structure):
    _fields_ = [("p", C.c_double), ("E0", C.c_double), ("Emin", C.c_double), ("nu", C.c_double)]


class tm_bcs(C.Structure):
    _fields_ = [("n", C.c_int64), ("dofs", C.POINTER(C.c_int64))]


class tm_options(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("n_geometric", C.c_int32), ("max_coarse", C.c_int32),
                ("smoother", C.c_int32), ("nu_pre", C.c_int32), ("nu_post", C.c_int32),
                ("omega", C.c_double), ("sa_beta", C.c_double), ("vcycle_fp", C.c_int32),
                ("outer", C.c_int32), ("max_iters", C.c_int32), ("check_every", C.c_int32),
                ("fine_mfma", C.c_int32), ("cheb_lower", C.c_double),
                ("adapt_iters", C.c_int32), ("cheb_warm_steps", C.c_int32),
                ("stencil_kernel", C.c_int32),
                ("sa_lds", C.c_int32), ("fine_tensor", C.c_int32)]


class tm_eig_options(C.Structure):
    _fields_ = [("nev", C.c_int32), ("j_min", C.c_int32), ("j_max", C.c_int32), ("max_iters", C.c_int32),
                ("tol", C.c_double), ("stag_tol", C.c_double), ("precond_fp", C.c_int32)]


# tm_allocator: device memory callbacks (alloc(bytes, stream, ctx), free(ptr, stream, ctx))
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class tm_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


def _torch_alloc(nbytes, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:           # out of memory: NULL, the library reports TM_ERR_OOM
        return None


def _torch_free(ptr, stream, ctx):
    torch.cuda.caching_allocator_delete(int(ptr))


# torch's caching allocator as the hierarchies' device memory (the callback
# objects live as long as the module)
TORCH_ALLOCATOR = tm_allocator(ALLOC_FN(_torch_alloc), FREE_FN(_torch_free), None)


class TmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libtopomg.so not built at {LIB_PATH}; run paper_2001_01655_amd.build")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    sig = {
        "tm_default_options": (None, [C.POINTER(tm_options)]),
        "tm_plan_bytes": (I32, [C.POINTER(tm_mesh), C.POINTER(tm_options), I32, C.POINTER(SZ)]),
        "tm_setup": (I32, [C.POINTER(tm_mesh), C.POINTER(tm_material), P, C.POINTER(tm_bcs),
                           C.POINTER(tm_options), C.POINTER(tm_allocator), P, C.POINTER(P)]),
        "tm_update_density": (I32, [P, P, P]),
        "tm_solve": (I32, [P, I32, P, D, I32, P, P, P, P, P]),
        "tm_solve_begin": (I32, [P, I32, P, D, I32, P, P, C.POINTER(P)]),
        "tm_solve_advance": (I32, [P, I32]),
        "tm_solve_poll": (I32, [P, C.POINTER(I32)]),
        "tm_batch_iterate": (I32, [I32, C.POINTER(P), I32, P]),
        "tm_solve_end": (I32, [P, P, P, P]),
        "tm_apply": (I32, [P, I32, I32, P, P, P]),
        "tm_vcycle": (I32, [P, I32, P, P, P]),
        "tm_level_info": (I32, [P, I32, C.POINTER(I64), C.POINTER(I64), C.POINTER(I32), C.POINTER(I32)]),
        "tm_num_levels": (I32, [P]),
        "tm_export_csr": (I32, [P, I32, P, P, P]),
        "tm_export_prolongator": (I32, [P, I32, C.POINTER(I64), C.POINTER(I64), P, P, P]),
        "tm_export_aggregates": (I32, [P, I32, P]),
        "tm_export_dinv": (I32, [P, I32, P]),
        "tm_export_coarse_inverse": (I32, [P, P]),
        "tm_export_connectivity": (I32, [C.POINTER(tm_mesh), P]),
        "tm_hierarchy_bytes": (I32, [P, C.POINTER(SZ)]),
        "tm_compliance_sensitivity": (I32, [P, I32, P, P, P]),
        "tm_density_filter": (I32, [C.POINTER(tm_mesh), D, I32, P, P, P]),
        "tm_density_filter_noalloc": (I32, [C.POINTER(tm_mesh), D, I32, P, P, P]),
        "tm_stress_stiffness": (I32, [P, P, D, P]),
        "tm_apply_stress_stiffness": (I32, [P, P, P, P]),
        "tm_default_eig_options": (None, [C.POINTER(tm_eig_options)]),
        "tm_eigs": (I32, [P, C.POINTER(tm_eig_options), I32, P, P, P, C.POINTER(I32), C.POINTER(I32), P]),
        "tm_kernel_timing": (I32, [P, I32, I32]),
        "tm_kernel_timing_read": (I32, [P, I32, C.POINTER(I64), C.POINTER(D)]),
        "tm_destroy": (None, [P]),
        "tm_status_string": (C.c_char_p, [I32]),
        "tm_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()
EXPORTED = [n for n in dir(LIB) if n.startswith("tm_")]


def check(status: int, what: str = "") -> int:
    """Raise TmError on a negative status; return the status otherwise."""
    if status < 0:
        msg = LIB.tm_last_error().decode() or LIB.tm_status_string(status).decode()
        raise TmError(status, f"{what}: {msg}" if what else msg)
    return status


def default_options(**kw) -> tm_options:
    o = tm_options()
    LIB.tm_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def default_eig_options(**kw) -> tm_eig_options:
    o = tm_eig_options()
    LIB.tm_default_eig_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def make_mesh(nel, h: float = 1.0) -> tm_mesh:
    m = tm_mesh()
    m.dim = len(nel)
    for i in range(3):
        m.nel[i] = int(nel[i]) if i < len(nel) else 1
    m.h = h
    return m


def make_material(p=3.0, E0=1.0, Emin=1e-9, nu=0.3) -> tm_material:
    return tm_material(p, E0, Emin, nu)


# thin C-named wrappers ------------------------------------------------------
def tm_plan_bytes(mesh: tm_mesh, opts: tm_options, n_rhs: int) -> int:
    b = C.c_size_t()
    check(LIB.tm_plan_bytes(C.byref(mesh), C.byref(opts), n_rhs, C.byref(b)), "tm_plan_bytes")
    return b.value


def tm_export_connectivity(mesh: tm_mesh):
    import numpy as np
    n_el = 1
    for i in range(mesh.dim):
        n_el *= mesh.nel[i]
    conn = np.empty((n_el, 2 ** mesh.dim), dtype=np.int32)
    check(LIB.tm_export_connectivity(C.byref(mesh), conn.ctypes.data), "tm_export_connectivity")
    return conn
