"""Oracle, part 6: the stress-stiffness matrix of the stability problem (CPU, FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Sec. 2 (stability maximisation) poses the generalized eigenproblem
K_sigma Phi = lambda K Phi with lambda_max = 1 / P_critical, and interpolates
the modulus that enters the stresses of K_sigma with its own law
E_sigma(rho) = E_max rho^p for rho >= 0.1 and 0 below.  The paper does not
write K_sigma out; this module takes the textbook linear-buckling definition
(the geometric or initial-stress stiffness of a continuum):

  * the stress of element e at a Gauss point g is
        sigma_g = E_sigma(rho_e) * C0 : eps(u_e)(g),
    C0 the unit-modulus isotropic law (plane stress in 2D), eps the small
    strain of the element's displacements;
  * the element's scalar geometric matrix is
        g_e[a, b] = sum_g w_g |J| grad N_a(g)^T sigma_g grad N_b(g),
    and it couples each displacement component with itself only, so the dof
    matrix is g_e (x) I_dim;
  * K_sigma = -sum_e L_e^T (g_e (x) I) L_e.  The minus sign makes compressive
    states give positive lambda (lambda = 1 / load factor), which is the sign
    the eigenproblem above needs;
  * Dirichlet conditions remove supported rows and columns:
        K_sigma~ = M K_sigma M   (no unit diagonal: K~ carries that one).

The 2x2(x2) Gauss rule integrates these element integrands exactly on square /
cube elements.  Parity of this construction with the paper is "as read": the
pins (tests) tie it to closed forms, to a tensor-product derivation of the
element integrals and to Euler's buckling load of a slender column.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import fem


def stress_modulus(rho: np.ndarray, p: float, E0: float, rho_min: float = 0.1) -> np.ndarray:
    """E_sigma(rho) = E0 rho^p where rho >= rho_min, else 0 (Sec. 2)."""
    rho = np.asarray(rho, dtype=np.float64)
    return np.where(rho >= rho_min, E0 * np.power(rho, p), 0.0)


def gauss_points(dim: int):
    g = 1.0 / np.sqrt(3.0)
    return [np.array(xi) for xi in itertools.product([-g, g], repeat=dim)]


def _voigt_to_tensor(dim: int, s: np.ndarray) -> np.ndarray:
    """Voigt stress (2D: xx, yy, xy; 3D: xx, yy, zz, yz, xz, xy) -> tensor."""
    if dim == 2:
        return np.array([[s[0], s[2]], [s[2], s[1]]])
    return np.array([[s[0], s[5], s[4]], [s[5], s[1], s[3]], [s[4], s[3], s[2]]])


def gauss_stresses(nel, u: np.ndarray, Es: np.ndarray, nu: float, h: float = 1.0) -> np.ndarray:
    """Stress tensors (n_el, 2^dim, dim, dim) at the Gauss points of every
    element, in the order of gauss_points, for displacements u (n_dof)."""
    dim = len(nel)
    D0 = fem.elasticity_matrix(dim, nu)
    ed = fem.element_dofs(nel)
    ue = u[ed]                                        # (n_el, dim * 2^dim)
    jac = h / 2.0
    out = np.zeros((ed.shape[0], 2 ** dim, dim, dim))
    for g, xi in enumerate(gauss_points(dim)):
        B = fem.strain_displacement(dim, fem._shape_grad_ref(dim, xi) / jac)
        sv = (ue @ B.T) @ D0.T                        # unit-modulus Voigt stress
        sv *= Es[:, None]
        for e in range(ed.shape[0]):
            out[e, g] = _voigt_to_tensor(dim, sv[e])
    return out


def element_geometric(dim: int, sig_gp: np.ndarray, h: float = 1.0) -> np.ndarray:
    """g[a, b] = sum_g w |J| grad N_a^T sigma_g grad N_b (2^dim x 2^dim), unit
    Gauss weights, |J| = (h/2)^dim (2D: unit thickness)."""
    jac = h / 2.0
    n = 2 ** dim
    G = np.zeros((n, n))
    for g, xi in enumerate(gauss_points(dim)):
        dN = fem._shape_grad_ref(dim, xi) / jac       # (n, dim)
        G += dN @ sig_gp[g] @ dN.T * jac ** dim
    return 0.5 * (G + G.T)      # symmetric by definition; drop rounding asymmetry


def stress_stiffness(nel, u: np.ndarray, rho: np.ndarray, p: float, E0: float, nu: float,
                     fixed: np.ndarray, h: float = 1.0, rho_min: float = 0.1) -> sp.csr_matrix:
    """K_sigma~ (CSR, n_dof x n_dof): minus the assembled geometric stiffness of
    the stresses of u, supported rows and columns removed."""
    dim = len(nel)
    Es = stress_modulus(rho, p, E0, rho_min)
    sig = gauss_stresses(nel, u, Es, nu, h)
    conn = fem.connectivity(nel)
    n = 2 ** dim
    rows, cols, vals = [], [], []
    for e in range(conn.shape[0]):
        g = element_geometric(dim, sig[e], h)
        for c in range(dim):
            r = dim * conn[e] + c
            rows.append(np.repeat(r, n))
            cols.append(np.tile(r, n))
            vals.append(-g.ravel())
    n_dof = dim * int(np.prod(fem.n_nodes_axis(nel)))
    Ks = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(n_dof, n_dof)).tocsr()
    Ks.sum_duplicates()
    m = sp.diags(fem.free_mask(n_dof, fixed))
    Ks = (m @ Ks @ m).tocsr()
    Ks.sort_indices()
    return Ks
