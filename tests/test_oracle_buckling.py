"""Pins of the oracle's stress-stiffness matrix (Sec. 2 stability problem, read
as the textbook geometric stiffness): Hooke's law in Lame form for uniform
strains, element integrals from 1D closed forms by tensor products, the
quadratic form of linear fields under a uniform stress, the translation null
space, the E_sigma cutoff, and Euler's load of a clamped-free column."""
import itertools

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import buckling, fem
from synth import problems as P


def _lame_stress(dim, eps, E, nu):
    if dim == 2:        # plane stress
        return E / (1 - nu * nu) * ((1 - nu) * eps + nu * np.trace(eps) * np.eye(2))
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return lam * np.trace(eps) * np.eye(3) + 2 * mu * eps


@pytest.mark.parametrize("nel,h", [((3, 2), 1.0), ((2, 3, 2), 0.5)])
def test_uniform_strain_gives_hookes_stress_everywhere(nel, h):
    dim = len(nel)
    rng = np.random.default_rng(1)
    G = rng.standard_normal((dim, dim))
    eps = 0.5 * (G + G.T)
    W = 0.5 * (G - G.T)                                # a rotation adds no stress
    X = fem.node_coordinates(nel, h)
    u = (X @ (eps + W).T).ravel()
    rho = rng.uniform(0.0, 1.0, int(np.prod(nel)))
    rho[0], rho[1] = 0.0999, 0.1
    Es = buckling.stress_modulus(rho, 3.0, 2.0)
    assert Es[0] == 0.0 and np.isclose(Es[1], 2.0 * 0.1 ** 3)
    S = buckling.gauss_stresses(nel, u, Es, 0.3, h)
    for e in range(len(rho)):
        want = _lame_stress(dim, eps, Es[e], 0.3)
        for g in range(2 ** dim):
            assert np.allclose(S[e, g], want, rtol=0, atol=1e-13 * (1 + abs(want).max()))


def _one_d(h):
    S = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h          # int N_a' N_b'
    M = h * np.array([[1 / 3, 1 / 6], [1 / 6, 1 / 3]])    # int N_a N_b
    C = np.array([[-0.5, -0.5], [0.5, 0.5]])              # int N_a' N_b
    return S, M, C


@pytest.mark.parametrize("dim,h", [(2, 1.0), (2, 3.0), (3, 1.0), (3, 0.5)])
def test_element_matrix_equals_tensor_products_of_1d_integrals(dim, h):
    rng = np.random.default_rng(dim)
    G = rng.standard_normal((dim, dim))
    sig = G + G.T
    g = buckling.element_geometric(dim, np.repeat(sig[None], 2 ** dim, axis=0), h)
    S, M, C = _one_d(h)
    loc = fem.local_nodes(dim)
    want = np.zeros((2 ** dim, 2 ** dim))
    for a, b in itertools.product(range(2 ** dim), repeat=2):
        for i, j in itertools.product(range(dim), repeat=2):
            t = 1.0
            for d in range(dim):
                pa, pb = loc[a, d], loc[b, d]
                if d == i and d == j:
                    t *= S[pa, pb]
                elif d == i:
                    t *= C[pa, pb]
                elif d == j:
                    t *= C[pb, pa]
                else:
                    t *= M[pa, pb]
            want[a, b] += sig[i, j] * t
    assert np.allclose(g, want, rtol=0, atol=1e-14 * abs(want).max())


@pytest.mark.parametrize("nel", [(4, 3), (3, 2, 2)])
def test_linear_fields_quadratic_form_and_translations(nel):
    dim = len(nel)
    rng = np.random.default_rng(7)
    G = rng.standard_normal((dim, dim))
    eps = 0.5 * (G + G.T)
    X = fem.node_coordinates(nel)
    u = (X @ eps.T).ravel()
    n_el = int(np.prod(nel))
    rho = np.ones(n_el)
    Ks = buckling.stress_stiffness(nel, u, rho, 3.0, 1.0, 0.3, np.array([], dtype=np.int64))
    sig = _lame_stress(dim, eps, 1.0, 0.3)
    A = rng.standard_normal((dim, dim))                 # field x_k = A[k] . X
    x = (X @ A.T).ravel()
    vol = float(n_el)
    assert np.isclose(x @ (Ks @ x), -vol * sum(A[k] @ sig @ A[k] for k in range(dim)), rtol=1e-12)
    for c in range(dim):
        t = np.zeros_like(x)
        t[c::dim] = 1.0
        assert np.abs(Ks @ t).max() < 1e-13 * abs(Ks).max()
    assert abs(Ks - Ks.T).max() <= 1e-15 * abs(Ks).max()


def test_supported_rows_and_columns_are_removed():
    p = P.small_case(2, (4, 3), seed=3)
    u = np.random.default_rng(0).standard_normal(p.n_dof)
    Ks = buckling.stress_stiffness(p.nel, u, p.rho, p.p, p.E0, p.nu, p.fixed).toarray()
    assert not Ks[p.fixed].any() and not Ks[:, p.fixed].any()


def test_euler_load_of_a_clamped_free_column():
    """lambda_max = 1 / P_cr for a unit load; Euler: P_cr = pi^2 E I / (4 L^2),
    I = b^3 / 12 (unit thickness).  8 x 96 square Q4 elements, E = 1."""
    p = P.column_2d(nel=(8, 96), uniform=True)
    KE = fem.element_stiffness(2, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    K = fem.apply_dirichlet(fem.assemble(p.nel, E, KE), p.fixed).toarray()
    u = sla.solve(K, p.loads[0], assume_a="pos")
    Ks = buckling.stress_stiffness(p.nel, u, p.rho, p.p, p.E0, p.nu, p.fixed).toarray()
    free = fem.free_mask(p.n_dof, p.fixed) > 0
    lam = sla.eigh(Ks[np.ix_(free, free)], K[np.ix_(free, free)], eigvals_only=True)
    b, L = p.nel
    pcr = np.pi ** 2 * (b ** 3 / 12.0) / (4.0 * L ** 2)
    assert abs(lam[-1] * pcr - 1.0) < 0.01
    assert abs(lam[-2] * 9.0 * pcr - 1.0) < 0.06          # second mode: 9 P_cr
