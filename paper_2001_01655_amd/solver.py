"""Python face of the C ABI for torch users: a Hierarchy owns one tm_hierarchy.

Marshalling only: tensors are passed to the library by device pointer on the
current torch stream; every step of setup and solve runs in libtopomg.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from ._lib import LIB, check


def _stream_ptr(stream: Optional[torch.cuda.Stream] = None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype=torch.float64) -> torch.Tensor:
    t = torch.as_tensor(t, dtype=dtype)
    if t.device.type != "cuda":
        t = t.to("cuda")
    return t.contiguous()


class SolveResult:
    def __init__(self, u, iters, compliance, relres, status):
        self.u = u
        self.iters = iters
        self.compliance = compliance
        self.relres = relres
        self.status = status

    @property
    def converged(self) -> bool:
        return self.status == L.TM_OK


class Hierarchy:
    """tm_setup / tm_update_density / tm_solve on one mesh, material and supports."""

    def __init__(self, nel: Sequence[int], rho, fixed, *, h: float = 1.0, p: float = 3.0,
                 E0: float = 1.0, Emin: float = 1e-9, nu: float = 0.3,
                 stream: Optional[torch.cuda.Stream] = None, allocator: Optional[str] = "torch", **options):
        """allocator: "torch" takes the hierarchy's device memory from torch's
        caching allocator; None lets the library use hipMalloc."""
        self.nel = tuple(int(n) for n in nel)
        self.dim = len(self.nel)
        self.mesh = L.make_mesh(self.nel, h)
        self.mat = L.make_material(p, E0, Emin, nu)
        self.opts = L.default_options(**options)
        self.n_nodes = int(np.prod([n + 1 for n in self.nel]))
        self.n_dof = self.dim * self.n_nodes
        self.n_el = int(np.prod(self.nel))
        rho_d = _dev(rho)
        if rho_d.numel() != self.n_el:
            raise ValueError("rho must hold one density per element")
        self._fixed = np.ascontiguousarray(np.asarray(fixed, dtype=np.int64).ravel())
        bcs = L.tm_bcs(len(self._fixed), self._fixed.ctypes.data_as(C.POINTER(C.c_int64)))
        hp = C.c_void_p()
        self._h = None
        if allocator not in ("torch", None):
            raise ValueError("allocator must be 'torch' or None")
        alloc = C.byref(L.TORCH_ALLOCATOR) if allocator == "torch" else None
        check(LIB.tm_setup(C.byref(self.mesh), C.byref(self.mat), C.c_void_p(rho_d.data_ptr()),
                           C.byref(bcs), C.byref(self.opts), alloc, _stream_ptr(stream), C.byref(hp)),
              "tm_setup")
        self._h = hp

    # ----------------------------------------------------------------- lifecycle
    def close(self):
        if self._h is not None:
            LIB.tm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    def update_density(self, rho, stream=None):
        """tm_update_density; returns without waiting for the device (its checks
        are reported by the next solve)."""
        rho_d = _dev(rho)
        if stream is not None:
            rho_d.record_stream(stream)      # read by the update's first kernel on that stream
        check(LIB.tm_update_density(self._h, C.c_void_p(rho_d.data_ptr()), _stream_ptr(stream)),
              "tm_update_density")

    # ----------------------------------------------------------------- solve
    def solve(self, f, rtol: float = 1e-8, u0=None, stream=None, out: Optional[torch.Tensor] = None) -> SolveResult:
        f_d = _dev(f)
        n_rhs = f_d.numel() // self.n_dof
        if n_rhs * self.n_dof != f_d.numel():
            raise ValueError("f must hold n_rhs * n_dof values")
        if u0 is not None:
            u = _dev(u0).clone() if out is None else out.copy_(_dev(u0))
        else:
            u = torch.empty_like(f_d) if out is None else out
        iters = (C.c_int32 * n_rhs)()
        comp = (C.c_double * n_rhs)()
        rel = (C.c_double * n_rhs)()
        st = check(LIB.tm_solve(self._h, n_rhs, C.c_void_p(f_d.data_ptr()), rtol, int(u0 is not None),
                                C.c_void_p(u.data_ptr()), iters, comp, rel, _stream_ptr(stream)), "tm_solve")
        return SolveResult(u.view(f_d.shape), list(iters), list(comp), list(rel), st)

    def begin(self, f, rtol: float, u0=None, stream=None):
        return SolveState(self, f, rtol, u0, stream)

    # ----------------------------------------------------------------- parity / inspection
    def num_levels(self) -> int:
        return LIB.tm_num_levels(self._h)

    def level_info(self, level: int):
        n, nnz, kind, bs = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32()
        check(LIB.tm_level_info(self._h, level, C.byref(n), C.byref(nnz), C.byref(kind), C.byref(bs)),
              "tm_level_info")
        return dict(n_rows=n.value, nnz=nnz.value, kind=kind.value, block=bs.value)

    def apply(self, level: int, x: torch.Tensor, fp: int = 64, stream=None) -> torch.Tensor:
        dt = torch.float64 if fp == 64 else torch.float32
        x = _dev(x, dt)
        y = torch.empty_like(x)
        check(LIB.tm_apply(self._h, level, fp, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                           _stream_ptr(stream)), "tm_apply")
        return y

    def vcycle(self, b: torch.Tensor, fp: int = 64, stream=None) -> torch.Tensor:
        dt = torch.float64 if fp == 64 else torch.float32
        b = _dev(b, dt)
        x = torch.empty_like(b)
        check(LIB.tm_vcycle(self._h, fp, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                            _stream_ptr(stream)), "tm_vcycle")
        return x

    def export_csr(self, level: int):
        info = self.level_info(level)
        n, nnz = info["n_rows"], info["nnz"]
        rp = np.empty(n + 1, np.int64)
        ci = np.empty(nnz, np.int32)
        v = np.empty(nnz, np.float64)
        check(LIB.tm_export_csr(self._h, level, rp.ctypes.data, ci.ctypes.data, v.ctypes.data),
              "tm_export_csr")
        return rp, ci, v

    def export_prolongator(self, level: int):
        n, nnz = C.c_int64(), C.c_int64()
        check(LIB.tm_export_prolongator(self._h, level, C.byref(n), C.byref(nnz), None, None, None),
              "tm_export_prolongator")
        rp = np.empty(n.value + 1, np.int64)
        ci = np.empty(nnz.value, np.int32)
        v = np.empty(nnz.value, np.float64)
        check(LIB.tm_export_prolongator(self._h, level, C.byref(n), C.byref(nnz), rp.ctypes.data,
                                        ci.ctypes.data, v.ctypes.data), "tm_export_prolongator")
        return rp, ci, v

    def export_aggregates(self, level: int) -> np.ndarray:
        info = self.level_info(level)
        a = np.empty(info["n_rows"] // info["block"], np.int32)
        check(LIB.tm_export_aggregates(self._h, level, a.ctypes.data), "tm_export_aggregates")
        return a

    def export_dinv(self, level: int) -> np.ndarray:
        info = self.level_info(level)
        bs = info["block"]
        d = np.empty((info["n_rows"] // bs, bs, bs), np.float64)
        check(LIB.tm_export_dinv(self._h, level, d.ctypes.data), "tm_export_dinv")
        return d

    def export_coarse_inverse(self) -> np.ndarray:
        n = self.level_info(self.num_levels() - 1)["n_rows"]
        a = np.empty((n, n), np.float64)
        check(LIB.tm_export_coarse_inverse(self._h, a.ctypes.data), "tm_export_coarse_inverse")
        return a

    def compliance_sensitivity(self, u, stream=None) -> torch.Tensor:
        """d(sum_k f_k^T u_k)/d rho_e for the solutions u (n_dof or (n_rhs, n_dof))."""
        u_d = _dev(u)
        n_rhs = u_d.numel() // self.n_dof
        if n_rhs * self.n_dof != u_d.numel() or n_rhs < 1:
            raise ValueError("u must hold whole solution vectors")
        dc = torch.empty(self.n_el, dtype=torch.float64, device=u_d.device)
        check(LIB.tm_compliance_sensitivity(self.handle, n_rhs, C.c_void_p(u_d.data_ptr()),
                                            C.c_void_p(dc.data_ptr()), _stream_ptr(stream)),
              "tm_compliance_sensitivity")
        return dc

    def stress_stiffness(self, u, rho_min: float = 0.1, stream=None):
        """tm_stress_stiffness: build K_sigma~ of the displacements u (n_dof)."""
        u_d = _dev(u)
        if u_d.numel() != self.n_dof:
            raise ValueError("u must hold one solution vector")
        check(LIB.tm_stress_stiffness(self.handle, C.c_void_p(u_d.data_ptr()), float(rho_min), _stream_ptr(stream)),
              "tm_stress_stiffness")

    def apply_stress_stiffness(self, x, stream=None) -> torch.Tensor:
        """y = K_sigma~ x with the matrix of the last stress_stiffness call."""
        x_d = _dev(x)
        if x_d.numel() != self.n_dof:
            raise ValueError("x must hold n_dof values")
        y = torch.empty_like(x_d)
        check(LIB.tm_apply_stress_stiffness(self.handle, C.c_void_p(x_d.data_ptr()), C.c_void_p(y.data_ptr()),
                                            _stream_ptr(stream)), "tm_apply_stress_stiffness")
        return y

    def eigs(self, v0, stream=None, want_vectors: bool = True, **opts):
        """tm_eigs: the largest eigenvalues of K_sigma~ Phi = lambda K~ Phi by
        generalized Davidson.  v0: (n_init, n_dof) start vectors.  Options as in
        tm_eig_options (nev, j_min, j_max, max_iters, tol, stag_tol, precond_fp).
        Returns (lambda (numpy, descending), Phi (nev, n_dof) or None, iters,
        n_conv, status)."""
        o = L.default_eig_options(**opts)
        v_d = _dev(v0)
        n_init = v_d.numel() // self.n_dof
        if n_init * self.n_dof != v_d.numel() or n_init < 1:
            raise ValueError("v0 must hold whole vectors")
        lam = np.zeros(max(1, o.nev))
        phi = torch.empty((o.nev, self.n_dof), dtype=torch.float64, device=v_d.device) if want_vectors else None
        it, nc = C.c_int32(), C.c_int32()
        st = check(LIB.tm_eigs(self.handle, C.byref(o), n_init, C.c_void_p(v_d.data_ptr()),
                               lam.ctypes.data_as(C.c_void_p),
                               C.c_void_p(phi.data_ptr()) if phi is not None else None,
                               C.byref(it), C.byref(nc), _stream_ptr(stream)), "tm_eigs")
        return lam[:o.nev], phi, it.value, nc.value, st

    def device_bytes(self) -> int:
        b = C.c_size_t()
        check(LIB.tm_hierarchy_bytes(self._h, C.byref(b)), "tm_hierarchy_bytes")
        return b.value

    def kernel_timing(self, cls: int, enable: bool):
        check(LIB.tm_kernel_timing(self._h, cls, int(enable)), "tm_kernel_timing")

    def kernel_timing_read(self, cls: int):
        n, ms = C.c_int64(), C.c_double()
        check(LIB.tm_kernel_timing_read(self._h, cls, C.byref(n), C.byref(ms)), "tm_kernel_timing_read")
        return n.value, ms.value


class SolveState:
    """tm_solve_begin / advance / poll / end for iteration-level scheduling."""

    def __init__(self, H: Hierarchy, f, rtol: float, u0=None, stream=None):
        self.H = H
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.f = _dev(f)
        self.n_rhs = self.f.numel() // H.n_dof
        self.u = _dev(u0).clone() if u0 is not None else torch.empty_like(self.f)
        sp = C.c_void_p()
        check(LIB.tm_solve_begin(H.handle, self.n_rhs, C.c_void_p(self.f.data_ptr()), rtol,
                                 int(u0 is not None), C.c_void_p(self.u.data_ptr()),
                                 _stream_ptr(self.stream), C.byref(sp)), "tm_solve_begin")
        self._st = sp
        self.result: Optional[SolveResult] = None

    @property
    def handle(self):
        return self._st

    def advance(self, k: int):
        check(LIB.tm_solve_advance(self._st, k), "tm_solve_advance")

    def poll(self) -> int:
        """1: every load case stopped; 0: enqueued iterations done, not stopped;
        -1: iterations still running."""
        d = C.c_int32()
        check(LIB.tm_solve_poll(self._st, C.byref(d)), "tm_solve_poll")
        return int(d.value)

    def end(self) -> SolveResult:
        if self.result is None:
            n = self.n_rhs
            iters = (C.c_int32 * n)()
            comp = (C.c_double * n)()
            rel = (C.c_double * n)()
            st = check(LIB.tm_solve_end(self._st, iters, comp, rel), "tm_solve_end")
            self._st = None
            self.result = SolveResult(self.u.view(self.f.shape), list(iters), list(comp), list(rel), st)
        return self.result


def tm_batch_iterate(states: Sequence[SolveState], k: int, stream: Optional[torch.cuda.Stream] = None):
    """k iterations of every state as grouped launches on `stream` (default:
    the current stream)."""
    arr = (C.c_void_p * len(states))(*[s.handle for s in states])
    check(LIB.tm_batch_iterate(len(states), arr, k, _stream_ptr(stream)), "tm_batch_iterate")


def density_filter(nel: Sequence[int], x, radius: float = 1.5, transpose: bool = False,
                   stream=None) -> torch.Tensor:
    """tm_density_filter: S x (or S^T x) for one value per element, S the linear
    density filter of the given radius in element sizes."""
    x_d = _dev(x)
    mesh = L.make_mesh(tuple(int(n) for n in nel))
    n_el = int(np.prod([int(n) for n in nel]))
    if x_d.numel() != n_el:
        raise ValueError("x must hold one value per element")
    out = torch.empty_like(x_d)
    check(LIB.tm_density_filter(C.byref(mesh), float(radius), int(bool(transpose)), C.c_void_p(x_d.data_ptr()),
                                C.c_void_p(out.data_ptr()), _stream_ptr(stream)), "tm_density_filter")
    return out
