"""Oracle, part 1: finite-element definitions (CPU, FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module;
only tests, the smoke check and the CPU-baseline leg of the benchmark use it.

Contents (each follows the paper's problem statement, Sec. 2, Eqs. for the
compliance problem and the modified SIMP law):
  * structured Q4 / Hex8 numbering and connectivity,
  * element stiffness KE of isotropic linear elasticity (plane stress, unit
    thickness, in 2D), integrated with 2x2(x2) Gauss points (exact here),
  * modified SIMP  E(rho) = Emin + (E0 - Emin) rho^p,
  * assembly K = sum_e E_e L_e^T KE L_e as CSR with the structural pattern
    (every pair of dofs whose nodes share an element; no zero dropping),
  * homogeneous Dirichlet conditions  K~ = M K M + (I - M)  (M = 0/1 mask of
    free dofs), so the solution is zero on supported dofs,
  * a matrix-free apply of K~ written straight from the element sum.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

# local node order: 2D counter-clockwise from the lower-left corner;
# 3D the bottom face (z = 0) counter-clockwise, then the top face.
LOCAL_2D = np.array([(0, 0), (1, 0), (1, 1), (0, 1)], dtype=np.int64)
LOCAL_3D = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
                     (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)], dtype=np.int64)


def local_nodes(dim: int) -> np.ndarray:
    return LOCAL_2D if dim == 2 else LOCAL_3D


def n_nodes_axis(nel):
    return [n + 1 for n in nel]


def node_index(nel, coords: np.ndarray) -> np.ndarray:
    """coords (..., dim) integer node coordinates -> node ids."""
    nx1 = nel[0] + 1
    ny1 = nel[1] + 1
    idx = coords[..., 0] + nx1 * coords[..., 1]
    if len(nel) == 3:
        idx = idx + nx1 * ny1 * coords[..., 2]
    return idx


def element_coords(nel) -> np.ndarray:
    """(n_el, dim) integer lower corner of every element, in element-id order."""
    grids = np.meshgrid(*[np.arange(n) for n in reversed(nel)], indexing="ij")
    return np.stack([g.ravel() for g in reversed(grids)], axis=1)


def connectivity(nel) -> np.ndarray:
    """(n_el, 2^dim) node ids of each element in local order."""
    dim = len(nel)
    base = element_coords(nel)
    return node_index(nel, base[:, None, :] + local_nodes(dim)[None, :, :])


def element_dofs(nel) -> np.ndarray:
    dim = len(nel)
    conn = connectivity(nel)
    return (dim * conn[:, :, None] + np.arange(dim)[None, None, :]).reshape(conn.shape[0], -1)


def node_coordinates(nel, h: float = 1.0) -> np.ndarray:
    grids = np.meshgrid(*[np.arange(n + 1) for n in reversed(nel)], indexing="ij")
    return h * np.stack([g.ravel() for g in reversed(grids)], axis=1).astype(np.float64)


# ------------------------------------------------------------------ material
def elasticity_matrix(dim: int, nu: float, E: float = 1.0) -> np.ndarray:
    """Voigt constitutive matrix. 2D: plane stress. 3D: strains ordered
    (xx, yy, zz, yz, xz, xy) with engineering shears."""
    if dim == 2:
        return E / (1.0 - nu * nu) * np.array([[1.0, nu, 0.0],
                                               [nu, 1.0, 0.0],
                                               [0.0, 0.0, (1.0 - nu) / 2.0]])
    c = E / ((1.0 + nu) * (1.0 - 2.0 * nu))
    D = np.zeros((6, 6))
    D[:3, :3] = nu
    np.fill_diagonal(D[:3, :3], 1.0 - nu)
    D[3, 3] = D[4, 4] = D[5, 5] = (1.0 - 2.0 * nu) / 2.0
    return c * D


def _shape_grad_ref(dim: int, xi: np.ndarray) -> np.ndarray:
    """Gradients of the (bi/tri)linear shape functions on [-1,1]^dim at xi.
    Returns (n_nodes, dim)."""
    s = 2.0 * local_nodes(dim) - 1.0          # node signs in reference coords
    g = np.zeros((len(s), dim))
    for a in range(len(s)):
        for d in range(dim):
            v = 1.0 / (2 ** dim)
            for e in range(dim):
                v *= s[a, e] if e == d else (1.0 + s[a, e] * xi[e])
            g[a, d] = v
    return g


def strain_displacement(dim: int, grad_phys: np.ndarray) -> np.ndarray:
    n = grad_phys.shape[0]
    if dim == 2:
        B = np.zeros((3, 2 * n))
        for a in range(n):
            dx, dy = grad_phys[a]
            B[0, 2 * a] = dx
            B[1, 2 * a + 1] = dy
            B[2, 2 * a] = dy
            B[2, 2 * a + 1] = dx
        return B
    B = np.zeros((6, 3 * n))
    for a in range(n):
        dx, dy, dz = grad_phys[a]
        B[0, 3 * a] = dx
        B[1, 3 * a + 1] = dy
        B[2, 3 * a + 2] = dz
        B[3, 3 * a + 1] = dz
        B[3, 3 * a + 2] = dy
        B[4, 3 * a] = dz
        B[4, 3 * a + 2] = dx
        B[5, 3 * a] = dy
        B[5, 3 * a + 1] = dx
    return B


def element_stiffness(dim: int, nu: float, h: float = 1.0) -> np.ndarray:
    """KE for E = 1 on a square / cube of edge h:  sum_gp B^T D B |J| w.
    Two Gauss points per axis integrate the affine-element integrand exactly.
    2D has unit thickness, so KE does not depend on h; in 3D KE scales with h."""
    D = elasticity_matrix(dim, nu)
    g = 1.0 / np.sqrt(3.0)
    jac = h / 2.0
    KE = np.zeros((dim * 2 ** dim, dim * 2 ** dim))
    for xi in itertools.product([-g, g], repeat=dim):
        grad = _shape_grad_ref(dim, np.array(xi)) / jac
        B = strain_displacement(dim, grad)
        KE += B.T @ D @ B * jac ** dim
    return 0.5 * (KE + KE.T)


def element_stiffness_box(dim: int, nu: float, sizes) -> np.ndarray:
    """KE for E = 1 on an axis-aligned box with the given edge lengths (the
    coarse elements of an odd-count coarsening are such boxes); equal to
    element_stiffness for a cube."""
    D = elasticity_matrix(dim, nu)
    g = 1.0 / np.sqrt(3.0)
    jac = np.asarray(sizes, dtype=float) / 2.0
    KE = np.zeros((dim * 2 ** dim, dim * 2 ** dim))
    for xi in itertools.product([-g, g], repeat=dim):
        grad = _shape_grad_ref(dim, np.array(xi)) / jac[None, :]
        B = strain_displacement(dim, grad)
        KE += B.T @ D @ B * np.prod(jac)
    return 0.5 * (KE + KE.T)


def simp(rho: np.ndarray, p: float, E0: float, Emin: float) -> np.ndarray:
    """Modified SIMP law  E = Emin + (E0 - Emin) rho^p."""
    return Emin + (E0 - Emin) * np.power(rho, p)


# ------------------------------------------------------------------ assembly
def assemble(nel, E: np.ndarray, KE: np.ndarray) -> sp.csr_matrix:
    """K = sum_e E_e L_e^T KE L_e as CSR (FP64), structural pattern, sorted columns."""
    ed = element_dofs(nel)
    nd = ed.shape[1]
    rows = np.repeat(ed, nd, axis=1).ravel()
    cols = np.tile(ed, (1, nd)).ravel()
    vals = (E[:, None, None] * KE[None, :, :]).ravel()
    n = len(nel) * int(np.prod(n_nodes_axis(nel)))
    K = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    return K


def free_mask(n_dof: int, fixed: np.ndarray) -> np.ndarray:
    m = np.ones(n_dof)
    m[np.asarray(fixed, dtype=np.int64)] = 0.0
    return m


def apply_dirichlet(K: sp.csr_matrix, fixed: np.ndarray) -> sp.csr_matrix:
    """K~ = M K M + (I - M): supported rows and columns keep only a unit diagonal."""
    m = free_mask(K.shape[0], fixed)
    C = K.tocoo()
    keep = ((m[C.row] > 0) & (m[C.col] > 0)) | (C.row == C.col)
    r, c, v = C.row[keep], C.col[keep], C.data[keep].copy()
    diag_fixed = (r == c) & (m[r] == 0)
    v[diag_fixed] = 1.0
    Kt = sp.csr_matrix((v, (r, c)), shape=K.shape)
    Kt.sort_indices()
    return Kt


def assemble_dirichlet_blocked(nel, E: np.ndarray, KE: np.ndarray, fixed: np.ndarray,
                               planes_per_block: int = 8) -> sp.csr_matrix:
    """K~ = M K M + (I - M) built in slabs of node planes along the slowest axis,
    so that only one slab's element contributions are held at a time (the
    one-shot assembly of a 5.4M-dof grid needs more host memory than a
    workstation has).  Each slab takes the element layers that touch its
    node planes, keeps the contributions whose row lies in the slab, drops the
    off-diagonal entries of supported rows and columns and puts a single unit
    diagonal on supported rows; the slabs are stacked in row order.  Every
    stored entry is the sum of the same element terms as in assemble() +
    apply_dirichlet()."""
    dim = len(nel)
    ed = element_dofs(nel)
    nd = ed.shape[1]
    n = dim * int(np.prod(n_nodes_axis(nel)))
    m = free_mask(n, fixed)
    plane_dofs = dim * int(np.prod([k + 1 for k in nel[:-1]]))
    el_layer = int(np.prod(nel[:-1]))
    n_planes = nel[-1] + 1
    blocks = []
    for p0 in range(0, n_planes, planes_per_block):
        p1 = min(p0 + planes_per_block, n_planes)
        e0, e1 = max(p0 - 1, 0) * el_layer, min(p1, nel[-1]) * el_layer
        sub = ed[e0:e1]
        rows = np.repeat(sub, nd, axis=1).ravel()
        cols = np.tile(sub, (1, nd)).ravel()
        vals = (E[e0:e1, None, None] * KE[None, :, :]).ravel()
        r0, r1 = p0 * plane_dofs, p1 * plane_dofs
        keep = (rows >= r0) & (rows < r1) & (m[rows] > 0) & (m[cols] > 0)
        rows, cols, vals = rows[keep], cols[keep], vals[keep]
        fx = np.nonzero(m[r0:r1] == 0)[0] + r0
        rows = np.concatenate([rows, fx])
        cols = np.concatenate([cols, fx])
        vals = np.concatenate([vals, np.ones(fx.shape[0])])
        B = sp.coo_matrix((vals, (rows - r0, cols)), shape=(r1 - r0, n)).tocsr()
        B.sum_duplicates()
        B.sort_indices()
        blocks.append(B)
        del rows, cols, vals, keep
    K = sp.vstack(blocks, format="csr")
    K.sort_indices()
    return K


def apply_matfree(nel, E: np.ndarray, KE: np.ndarray, fixed: np.ndarray,
                  x: np.ndarray, chunk: int = 1 << 18) -> np.ndarray:
    """y = K~ x = M (sum_e E_e L_e^T KE L_e) M x + (I - M) x, element by element."""
    ed = element_dofs(nel)
    m = free_mask(x.shape[0], fixed)
    xm = m * x
    y = np.zeros_like(x)
    for s in range(0, ed.shape[0], chunk):
        e = ed[s:s + chunk]
        ue = xm[e]
        ye = E[s:s + chunk, None] * (ue @ KE.T)
        y += np.bincount(e.ravel(), weights=ye.ravel(), minlength=y.shape[0])
    return m * y + (1.0 - m) * x


def rigid_body_modes(coords: np.ndarray) -> np.ndarray:
    """Near-nullspace of unconstrained elasticity at the given node coordinates,
    rows per node interleaved by component. 2D: e_x, e_y, (-y, x).
    3D: e_x, e_y, e_z, (0, -z, y), (z, 0, -x), (-y, x, 0)."""
    n, dim = coords.shape
    if dim == 2:
        B = np.zeros((n, 2, 3))
        B[:, 0, 0] = 1.0
        B[:, 1, 1] = 1.0
        B[:, 0, 2] = -coords[:, 1]
        B[:, 1, 2] = coords[:, 0]
        return B.reshape(2 * n, 3)
    x, y, z = coords[:, 0], coords[:, 1], coords[:, 2]
    B = np.zeros((n, 3, 6))
    B[:, 0, 0] = B[:, 1, 1] = B[:, 2, 2] = 1.0
    B[:, 1, 3] = -z
    B[:, 2, 3] = y
    B[:, 0, 4] = z
    B[:, 2, 4] = -x
    B[:, 0, 5] = -y
    B[:, 1, 5] = x
    return B.reshape(3 * n, 6)


# ------------------------------------------------------------- sensitivities
def compliance_sensitivity(nel, rho: np.ndarray, p: float, E0: float, Emin: float, KE: np.ndarray,
                           U: np.ndarray) -> np.ndarray:
    """d/d rho_e of sum_k c_k, c_k = f_k^T u_k, for the modified SIMP law (Sec. 2):
    compliance is self-adjoint, so dc_k/d rho_e = -u_k,e^T (dK/d rho_e) u_k,e with
    dK/d rho_e = p rho_e^(p-1) (E0 - Emin) L_e^T KE L_e.  U holds the solutions
    (n_rhs, n_dof), zero on supported dofs."""
    ed = element_dofs(nel)
    dE = p * np.power(rho, p - 1.0) * (E0 - Emin)
    U = np.atleast_2d(U)
    q = np.zeros(ed.shape[0])
    for u in U:
        ue = u[ed]
        q += np.einsum("ei,ij,ej->e", ue, KE, ue)
    return -dE * q
