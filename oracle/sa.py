"""Oracle, part 3: smoothed-aggregation coarse levels and the GMG->AMG hybrid
(CPU, FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Follows Sec. 3.2 (algebraic multigrid: strength of connection, aggregation into
supernodes, restriction, Galerkin projection), Sec. 4 (block strength of
connection with beta = 0.003, one value per node; the tentative prolongator
improved by a weighted-Jacobi step; rigid-body modes as candidates) and the
hybrid of Sec. 4.3 / 4.4 (geometric restrictions on the finest levels, then
algebraic coarsening to a coarse-size limit).

Readings (the paper does not fix these):
  * block strength: with f_IJ the squared Frobenius norm of block (I, J),
    I != J is strong iff f_IJ^2 > beta^2 f_II f_JJ; the graph is symmetrised;
  * aggregation: see agg.c (lexicographically-first maximal distance-2
    independent set under a hashed key, then two joining passes);
  * near-nullspace: rigid-body modes at the node coordinates of the level the
    algebraic coarsening starts from, columns translations then rotations;
  * tentative prolongator: per aggregate, modified Gram-Schmidt in column
    order with R_jj >= 0; a column whose remaining norm is <= 1e-10 of its
    original norm is set to zero but kept in the pattern;
  * smoothed prolongator P = T - omega D^-1 A T with D the point-block diagonal
    and omega = (4/3) / ||D^-1 A||_inf;
  * stop when the level has fewer than max_coarse dofs, or when a coarsening
    step keeps more than 90% of the dofs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp

from . import fem, mg

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def build_c(force: bool = False) -> str:
    """Compile agg.c into a shared object next to it."""
    so = os.path.join(_HERE, "_agg.so")
    src = os.path.join(_HERE, "agg.c")
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", src, "-o", so])
    return so


def _lib():
    global _LIB
    if _LIB is None:
        _LIB = ctypes.CDLL(build_c())
        _LIB.oracle_aggregate.restype = ctypes.c_int64
        _LIB.oracle_aggregate.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]
        _LIB.oracle_fmix32.restype = ctypes.c_uint32
        _LIB.oracle_fmix32.argtypes = [ctypes.c_uint32]
    return _LIB


def fmix32(i: int) -> int:
    return int(_lib().oracle_fmix32(ctypes.c_uint32(i)))


# ------------------------------------------------------------ strength
def block_sq_norms(A: sp.csr_matrix, bs: int) -> sp.csr_matrix:
    """Node-level matrix of squared Frobenius norms of the bs x bs blocks."""
    C = A.tocoo()
    nb = A.shape[0] // bs
    F = sp.coo_matrix((C.data * C.data, (C.row // bs, C.col // bs)), shape=(nb, nb)).tocsr()
    F.sum_duplicates()
    F.sort_indices()
    return F


def strength(A: sp.csr_matrix, bs: int, beta: float = 0.003) -> sp.csr_matrix:
    """Symmetric node strength graph (no self loops) as a 0/1 CSR matrix."""
    F = block_sq_norms(A, bs)
    d = F.diagonal()
    Fc = F.tocoo()
    off = Fc.row != Fc.col
    r, c, f = Fc.row[off], Fc.col[off], Fc.data[off]
    strong = f * f > (beta * beta) * (d[r] * d[c])
    S = sp.coo_matrix((np.ones(strong.sum()), (r[strong], c[strong])), shape=F.shape).tocsr()
    S = ((S + S.T) > 0).astype(np.float64).tocsr()
    S.sort_indices()
    return S


def aggregate(S: sp.csr_matrix):
    """(agg[n] int32, is_root[n] bool, n_agg)."""
    n = S.shape[0]
    rowptr = np.ascontiguousarray(S.indptr, dtype=np.int64)
    col = np.ascontiguousarray(S.indices, dtype=np.int32)
    agg = np.empty(n, dtype=np.int32)
    root = np.empty(n, dtype=np.uint8)
    n_agg = _lib().oracle_aggregate(n, rowptr.ctypes.data, col.ctypes.data,
                                    agg.ctypes.data, root.ctypes.data)
    if n_agg < 0:
        raise RuntimeError("aggregation left nodes unassigned")
    return agg, root.astype(bool), int(n_agg)


# ------------------------------------------------------------ prolongators
def tentative(agg: np.ndarray, n_agg: int, B: np.ndarray, bs: int):
    """T (n_dof x n_agg*k) and coarse candidates Bc (n_agg*k x k) by per-aggregate
    modified Gram-Schmidt of the candidate rows."""
    n_nodes = agg.shape[0]
    k = B.shape[1]
    members = [[] for _ in range(n_agg)]
    for i in range(n_nodes):
        members[agg[i]].append(i)
    rows, cols, vals = [], [], []
    Bc = np.zeros((n_agg * k, k))
    for g in range(n_agg):
        nodes = np.array(members[g], dtype=np.int64)
        dofs = (bs * nodes[:, None] + np.arange(bs)[None, :]).ravel()
        V = B[dofs, :].copy()
        Q = np.zeros_like(V)
        R = np.zeros((k, k))
        for j in range(k):
            v = V[:, j].copy()
            n0 = np.linalg.norm(v)
            for i in range(j):
                R[i, j] = Q[:, i] @ v
                v = v - R[i, j] * Q[:, i]
            nr = np.linalg.norm(v)
            if n0 == 0.0 or nr <= 1e-10 * n0:
                R[j, j] = 0.0
            else:
                R[j, j] = nr
                Q[:, j] = v / nr
        rr = np.repeat(dofs, k)
        cc = np.tile(g * k + np.arange(k), dofs.shape[0])
        rows.append(rr)
        cols.append(cc)
        vals.append(Q.ravel())
        Bc[g * k:(g + 1) * k] = R
    T = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(bs * n_nodes, n_agg * k))
    T.sort_indices()
    return T, Bc


def jacobi_weight(A: sp.csr_matrix, Dinv: sp.csr_matrix) -> float:
    """omega = (4/3) / ||D^-1 A||_inf."""
    DA = mg.structural_matmul(Dinv, A)
    lam = np.max(np.asarray(abs(DA).sum(axis=1)).ravel())
    return (4.0 / 3.0) / lam


def smoothed_prolongator(A: sp.csr_matrix, T: sp.csr_matrix, bs: int) -> sp.csr_matrix:
    Dinv = mg.block_diag_inverse(A, bs)
    w = jacobi_weight(A, Dinv)
    DAT = mg.structural_matmul(Dinv, mg.structural_matmul(A, T))
    return mg.structural_add(T, -w * DAT)


# ------------------------------------------------------------ hybrid
def level_node_positions(nel, levels: int, h: float = 1.0):
    """Element counts and per-axis physical node positions of geometric level
    levels - 1 (the fine grid is level 0): each coarsening takes n elements to
    ceil(n/2) and puts coarse node I on fine node min(2I, n) of the level
    above, so an odd count leaves a last coarse element of one fine element."""
    pos = [h * np.arange(n + 1, dtype=np.float64) for n in nel]
    cur = list(nel)
    for _ in range(levels - 1):
        nxt = [mg.coarse_count(n) for n in cur]
        pos = [p[np.minimum(2 * np.arange(m + 1), n)] for p, m, n in zip(pos, nxt, cur)]
        cur = nxt
    return cur, pos


def build_hybrid(nel, E, KE, fixed, n_geometric: int, max_coarse: int = 1000,
                 beta: float = 0.003, omega: float = 0.5, nu_pre: int = 1, nu_post: int = 1,
                 h: float = 1.0, smoother: str = "jacobi", cheb_lower: float = 0.1) -> mg.Hierarchy:
    """n_geometric levels (fine grid included) of geometric coarsening, then
    smoothed aggregation until the level has fewer than max_coarse dofs."""
    dim = len(nel)
    Hg = mg.build_geometric(nel, E, KE, fixed, n_geometric, omega, nu_pre, nu_post)
    As, Ps, bss, kinds = list(Hg.A), list(Hg.P), list(Hg.bs), list(Hg.kinds)
    aggs = [None] * len(As)
    _, pos = level_node_positions(nel, n_geometric, h)
    grids = np.meshgrid(*[pos[d] for d in reversed(range(dim))], indexing="ij")
    coords = np.stack([g.ravel() for g in reversed(grids)], axis=1)
    Bcand = fem.rigid_body_modes(coords)
    A, bs = As[-1], dim
    while A.shape[0] >= max_coarse:
        S = strength(A, bs, beta)
        agg, _, n_agg = aggregate(S)
        T, Bc = tentative(agg, n_agg, Bcand, bs)
        P = smoothed_prolongator(A, T, bs)
        if P.shape[1] > 0.9 * A.shape[0]:
            break
        Ac = mg.galerkin(P, A)
        aggs[-1] = agg
        Ps.append(P)
        As.append(Ac)
        aggs.append(None)
        kinds.append("sa")
        bs = Bcand.shape[1]
        bss.append(bs)
        A, Bcand = Ac, Bc
    return mg.finish(As, Ps, bss, omega, nu_pre, nu_post, False, kinds, aggs, smoother=smoother,
                     cheb_lower=cheb_lower, fixed=fixed)
