"""Oracle, part 2: multigrid-preconditioned CG on assembled CSR (CPU, FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Follows the paper's Sec. 3 (Solvers):
  * geometric prolongation P from the shape functions of the coarse grid
    (bilinear / trilinear), restriction R = P^T, Galerkin coarse operators
    A^{i+1} = P^T A^i P  (the Galerkin-projection equation of Sec. 3.2);
  * the V-cycle of Algorithm 1 with weighted (point-block) Jacobi smoothing,
    read as the standard recursion (the coarsest branch solves with the
    coarsest operator; see the readings listed beside the oracle);
  * the coarsest operator factorised once at setup (dense Cholesky here);
  * conjugate gradients preconditioned by one V-cycle (Sec. 3.1).

Readings of the paper that this code fixes (the paper is silent on them):
  * coarse node I sits on fine node 2I; weights per axis w(0)=1, w(+-1)=1/2;
  * supported fine dofs are dropped from P on level 0 (P~ = M P); coarse
    levels carry no supports;
  * a dof whose Galerkin diagonal is exactly zero gets a unit diagonal;
  * "n levels" counts the fine grid; automatic level count stops at the first
    level with fewer than `max_coarse` dofs.
No zero dropping happens anywhere: every sparse product keeps its structural
pattern.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem


# ------------------------------------------------------------ level planning
def level_dofs(nel, L: int, ceil: bool = False) -> List[int]:
    """dofs of levels 0..L-1 when each level halves the element counts
    (ceil(n/2) for odd counts if `ceil`); constrained dofs are counted."""
    out = []
    cur = list(nel)
    for _ in range(L):
        out.append(len(nel) * int(np.prod([n + 1 for n in cur])))
        cur = [(n + 1) // 2 if ceil else n // 2 for n in cur]
    return out


def plan_levels(nel, n_levels: int = 0, max_coarse: int = 1000) -> int:
    """Number of geometric levels (fine grid included).  n_levels > 0 is taken
    as given; otherwise coarsen while the current level has >= max_coarse dofs
    and every element count is even."""
    if n_levels > 0:
        return n_levels
    L = 1
    cur = list(nel)
    while len(nel) * int(np.prod([n + 1 for n in cur])) >= max_coarse and all(n % 2 == 0 and n >= 2 for n in cur):
        cur = [n // 2 for n in cur]
        L += 1
    return L


# ------------------------------------------------------------ sparse helpers
def _ones(A: sp.csr_matrix) -> sp.csr_matrix:
    B = A.copy().tocsr()
    B.data = np.ones_like(B.data)
    return B


def structural_matmul(A: sp.spmatrix, B: sp.spmatrix) -> sp.csr_matrix:
    """A @ B with the structural pattern (entries that cancel to zero are kept)."""
    A = sp.csr_matrix(A)
    B = sp.csr_matrix(B)
    S = (_ones(A) @ _ones(B)).tocsr()       # positive sums never cancel
    S.sort_indices()
    C = (A @ B).tocsr()
    C.sort_indices()
    out = S.copy()
    out.data = np.zeros_like(out.data, dtype=np.float64)
    # scatter C's stored values into S's pattern
    Cc = C.tocoo()
    rows_S = np.repeat(np.arange(S.shape[0]), np.diff(S.indptr))
    keyS = rows_S.astype(np.int64) * S.shape[1] + S.indices
    keyC = Cc.row.astype(np.int64) * S.shape[1] + Cc.col
    pos = np.searchsorted(keyS, keyC)
    out.data[pos] = Cc.data
    return out


def structural_add(A: sp.spmatrix, B: sp.spmatrix) -> sp.csr_matrix:
    """A + B on the union of the two patterns (no zero dropping)."""
    A = sp.csr_matrix(A)
    B = sp.csr_matrix(B)
    S = (_ones(A) + _ones(B)).tocsr()
    S.sort_indices()
    out = S.copy()
    out.data = np.zeros_like(out.data, dtype=np.float64)
    rows_S = np.repeat(np.arange(S.shape[0]), np.diff(S.indptr))
    keyS = rows_S.astype(np.int64) * S.shape[1] + S.indices
    for M in (A, B):
        Mc = M.tocoo()
        key = Mc.row.astype(np.int64) * S.shape[1] + Mc.col
        np.add.at(out.data, np.searchsorted(keyS, key), Mc.data)
    return out


def galerkin(P: sp.spmatrix, A: sp.spmatrix, block_rows: Optional[int] = None) -> sp.csr_matrix:
    """A_c = P^T (A P), structural pattern; exactly-zero diagonals set to 1.
    With `block_rows`, the product is summed over row blocks b of A and P,
    A_c = sum_b P_b^T (A_b P), so that only one block's A P is held at a time
    (same pattern; the sums are associated by block)."""
    if block_rows is None or block_rows >= A.shape[0]:
        Ac = structural_matmul(sp.csr_matrix(P.T), structural_matmul(A, P))
    else:
        A = sp.csr_matrix(A)
        P = sp.csr_matrix(P)
        Ac = None
        for r0 in range(0, A.shape[0], block_rows):
            r1 = min(r0 + block_rows, A.shape[0])
            part = structural_matmul(sp.csr_matrix(P[r0:r1].T), structural_matmul(A[r0:r1], P))
            Ac = part if Ac is None else structural_add(Ac, part)
    d = Ac.diagonal()
    if np.any(d == 0.0):
        Ac = Ac.tolil()
        for i in np.nonzero(d == 0.0)[0]:
            Ac[i, i] = 1.0
        Ac = Ac.tocsr()
    Ac.sort_indices()
    return Ac


# ------------------------------------------------------- geometric transfers
def coarse_count(n: int) -> int:
    """Elements of the next coarser level along an axis: ceil(n/2) (Sec. 4.3)."""
    return (n + 1) // 2


def axis_prolongator(n: int) -> sp.csr_matrix:
    """1D interpolation from the coarse nodes (ceil(n/2) elements) to the n + 1
    fine nodes of one axis.  Coarse node I sits on fine node min(2I, n): a fine
    node on a coarse node takes it with weight 1, a fine node halfway between two
    coarse nodes takes each with weight 1/2 (for odd n the last coarse element is
    one fine element, so its end nodes are both coarse)."""
    nc = coarse_count(n)
    pos = np.minimum(2 * np.arange(nc + 1), n)
    W = np.zeros((n + 1, nc + 1))
    for I, x in enumerate(pos):
        W[x, I] = 1.0
    for i in range(n + 1):
        if W[i].sum() == 0.0:                      # strictly between two coarse nodes
            left = np.searchsorted(pos, i) - 1
            W[i, left] = W[i, left + 1] = 0.5
    return sp.csr_matrix(W)


def geometric_prolongator(nel, fixed: Optional[np.ndarray] = None) -> sp.csr_matrix:
    """P (fine dofs x coarse dofs) from coarse-grid shape functions: the tensor
    product of the per-axis interpolations (x fastest), identity over the dof
    components.  If `fixed` is given, the rows of supported fine dofs are
    dropped (P~ = M P)."""
    dim = len(nel)
    Pn = axis_prolongator(nel[0])
    for n in nel[1:]:
        Pn = sp.kron(axis_prolongator(n), Pn, format="csr")     # slower axes to the left
    P = sp.kron(Pn, sp.identity(dim), format="csr")
    P.eliminate_zeros()
    if fixed is not None and len(fixed) > 0:
        m = fem.free_mask(P.shape[0], fixed)
        P = sp.diags(m) @ P
        P.eliminate_zeros()
    P = sp.csr_matrix(P)
    P.sort_indices()
    return P


# ----------------------------------------------------------- smoothers
def block_diag_inverse(A: sp.csr_matrix, bs: int) -> sp.csr_matrix:
    """Inverse of the point-block diagonal of A (blocks of bs x bs) as a
    block-diagonal CSR matrix."""
    n = A.shape[0]
    nb = n // bs
    blocks = np.zeros((nb, bs, bs))
    C = A.tocoo()
    same = (C.row // bs) == (C.col // bs)
    blocks[C.row[same] // bs, C.row[same] % bs, C.col[same] % bs] = C.data[same]
    inv = np.linalg.inv(blocks)
    base = np.arange(nb)[:, None, None] * bs
    r = np.broadcast_to(base + np.arange(bs)[None, :, None], (nb, bs, bs))
    c = np.broadcast_to(base + np.arange(bs)[None, None, :], (nb, bs, bs))
    Dinv = sp.csr_matrix((inv.ravel(), (r.ravel(), c.ravel())), shape=(n, n))
    Dinv.sort_indices()
    return Dinv


def point_diag_inverse(A: sp.csr_matrix) -> sp.csr_matrix:
    return sp.diags(1.0 / A.diagonal()).tocsr()


# ----------------------------------------------------------- hierarchy
@dataclass
class Hierarchy:
    A: List[sp.csr_matrix]                 # level operators (A[0] = K~)
    P: List[sp.csr_matrix]                 # P[l]: level l+1 -> level l
    Dinv: List[sp.csr_matrix]              # smoother block inverses per level
    bs: List[int]                          # block size per level
    omega: float
    nu_pre: int
    nu_post: int
    chol: Optional[tuple] = None           # factor of the coarsest operator
    kinds: List[str] = field(default_factory=list)   # 'geo' or 'sa' per transfer
    aggregates: List[Optional[np.ndarray]] = field(default_factory=list)
    info: dict = field(default_factory=dict)
    smoother: str = "jacobi"               # 'jacobi' or 'chebyshev'
    cheb: List[Optional[tuple]] = field(default_factory=list)   # (theta, delta) per level

    @property
    def L(self) -> int:
        return len(self.A)


def build_geometric(nel, E: np.ndarray, KE: np.ndarray, fixed: np.ndarray, L: int,
                    omega: float = 0.5, nu_pre: int = 1, nu_post: int = 1,
                    point_jacobi: bool = False, smoother: str = "jacobi",
                    cheb_lower: float = 0.1, lean: bool = False) -> Hierarchy:
    """Pure geometric hierarchy with L levels (fine grid included).  `lean`
    assembles K~ in slabs and forms the Galerkin products in row blocks (same
    operators, for grids whose one-shot products do not fit in host memory)."""
    dim = len(nel)
    if lean:
        A0 = fem.assemble_dirichlet_blocked(nel, E, KE, fixed)
    else:
        A0 = fem.apply_dirichlet(fem.assemble(nel, E, KE), fixed)
    As, Ps = [A0], []
    cur = list(nel)
    for l in range(L - 1):
        if any(n < 2 for n in cur):
            raise ValueError(f"element counts {cur} cannot be coarsened at level {l}")
        P = geometric_prolongator(tuple(cur), fixed if l == 0 else None)
        Ps.append(P)
        As.append(galerkin(P, As[-1], block_rows=(1 << 20) if lean else None))
        cur = [coarse_count(n) for n in cur]
    return finish(As, Ps, [dim] * L, omega, nu_pre, nu_post, point_jacobi, ["geo"] * (L - 1),
                  smoother=smoother, cheb_lower=cheb_lower, fixed=fixed)


def finish(As, Ps, bss, omega, nu_pre, nu_post, point_jacobi=False, kinds=None,
           aggregates=None, smoother="jacobi", cheb_lower=0.1, fixed=None) -> Hierarchy:
    Dinv = [point_diag_inverse(A) if point_jacobi else block_diag_inverse(A, b)
            for A, b in zip(As, bss)]
    Ac = As[-1].toarray()
    chol = sla.cho_factor(Ac, lower=True)
    cheb = [None] * len(As)
    if smoother == "chebyshev":
        for l in range(len(As) - 1):
            mask = None
            if l == 0 and fixed is not None:
                mask = fem.free_mask(As[0].shape[0], fixed)
            lam = power_lmax(As[l], Dinv[l], mask)
            a, b = cheb_lower * lam, 1.1 * lam
            cheb[l] = ((b + a) / 2.0, (b - a) / 2.0)
    return Hierarchy(As, Ps, Dinv, list(bss), omega, nu_pre, nu_post, chol,
                     kinds or [], aggregates or [None] * len(As), smoother=smoother, cheb=cheb)


# ----------------------------------------------------------- Chebyshev smoothing
def _fmix32(x: np.ndarray) -> np.ndarray:
    """MurmurHash3's 32-bit finaliser (a published bijection of uint32)."""
    x = np.asarray(x, dtype=np.uint64) & 0xFFFFFFFF
    x ^= x >> 16
    x = (x * 0x85EBCA6B) & 0xFFFFFFFF
    x ^= x >> 13
    x = (x * 0xC2B2AE35) & 0xFFFFFFFF
    x ^= x >> 16
    return x


def power_start(n: int) -> np.ndarray:
    """Deterministic start vector: v_i = 1 + (fmix32(i) mod 2^16) / 2^16."""
    return 1.0 + (_fmix32(np.arange(n)) & 0xFFFF).astype(np.float64) / 65536.0


def power_lmax(A: sp.csr_matrix, Dinv: sp.csr_matrix, mask: Optional[np.ndarray] = None,
               iters: int = 12) -> float:
    """Estimate of the largest eigenvalue of D^-1 A by `iters` power steps from
    power_start (zero on supported dofs when a mask is given):
    lambda = ||D^-1 A v|| / ||v||, v <- D^-1 A v / ||D^-1 A v||."""
    v = power_start(A.shape[0])
    if mask is not None:
        v = v * mask
    lam = 0.0
    for _ in range(iters):
        z = Dinv @ (A @ v)
        nz, nv = np.linalg.norm(z), np.linalg.norm(v)
        lam = nz / nv
        v = z / nz
    return float(lam)


def chebyshev_smooth(A, Dinv, b, x, theta: float, delta: float, nu: int) -> np.ndarray:
    """nu steps of Chebyshev iteration for D^-1 A on the interval
    [theta - delta, theta + delta] (three-term recurrence):
    d_0 = D^-1 r_0 / theta, rho_0 = delta / theta;
    rho_k = 1 / (2 theta / delta - rho_{k-1}),
    d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / delta) D^-1 r_k;  x <- x + d_k.
    The residual after nu steps is T_nu((theta - D^-1 A) / delta) / T_nu(theta / delta)
    applied to the initial one."""
    sigma = theta / delta
    rho = 1.0 / sigma
    d = (Dinv @ (b - A @ x)) / theta
    x = x + d
    for _ in range(1, nu):
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (Dinv @ (b - A @ x))
        x = x + d
        rho = rho_new
    return x


# ----------------------------------------------------------- V-cycle
def vcycle(H: Hierarchy, b: np.ndarray, level: int = 0) -> np.ndarray:
    """Algorithm 1 (standard recursion): zero start, nu_pre weighted block-Jacobi
    sweeps, restrict the residual with P^T, recurse (or solve exactly on the
    coarsest level), prolongate and add, nu_post sweeps."""
    if level == H.L - 1:
        return sla.cho_solve(H.chol, b)
    A, Dinv, w = H.A[level], H.Dinv[level], H.omega
    x = np.zeros_like(b)
    if H.smoother == "chebyshev":
        th, de = H.cheb[level]
        x = chebyshev_smooth(A, Dinv, b, x, th, de, H.nu_pre)
    else:
        for _ in range(H.nu_pre):
            x = x + w * (Dinv @ (b - A @ x))
    bc = H.P[level].T @ (b - A @ x)
    x = x + H.P[level] @ vcycle(H, bc, level + 1)
    if H.smoother == "chebyshev":
        x = chebyshev_smooth(A, Dinv, b, x, th, de, H.nu_post)
    else:
        for _ in range(H.nu_post):
            x = x + w * (Dinv @ (b - A @ x))
    return x


# ----------------------------------------------------------- PCG
@dataclass
class SolveResult:
    u: np.ndarray
    iters: int
    relres: float            # recursive residual / ||f||
    true_relres: float       # ||f - K u|| / ||f||
    compliance: float
    converged: bool
    history: List[float] = field(default_factory=list)


def pcg(apply_A, precond, f: np.ndarray, rtol: float, u0: Optional[np.ndarray] = None,
        max_iters: int = 5000) -> SolveResult:
    """Preconditioned conjugate gradients (Hestenes-Stiefel form).  Stops when the
    recursive residual satisfies ||r_k|| <= rtol ||f||."""
    u = np.zeros_like(f) if u0 is None else u0.copy()
    r = f - apply_A(u) if u0 is not None else f.copy()
    nf = np.linalg.norm(f)
    if nf == 0.0:
        return SolveResult(u, 0, 0.0, 0.0, 0.0, True)
    hist = [np.linalg.norm(r) / nf]
    z = precond(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while hist[-1] > rtol and it < max_iters:
        q = apply_A(p)
        alpha = rz / (p @ q)
        u = u + alpha * p
        r = r - alpha * q
        it += 1
        hist.append(np.linalg.norm(r) / nf)
        if hist[-1] <= rtol:
            break
        z = precond(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    true = np.linalg.norm(f - apply_A(u)) / nf
    return SolveResult(u, it, hist[-1], true, float(f @ u), hist[-1] <= rtol, hist)


def mg_pcg(H: Hierarchy, f: np.ndarray, rtol: float, u0=None, max_iters: int = 5000) -> SolveResult:
    A0 = H.A[0]
    return pcg(lambda v: A0 @ v, lambda r: vcycle(H, r), f, rtol, u0, max_iters)


def dense_solve(A: sp.spmatrix, f: np.ndarray) -> np.ndarray:
    """Direct solve by dense Cholesky (small systems only)."""
    return sla.cho_solve(sla.cho_factor(A.toarray(), lower=True), f)
