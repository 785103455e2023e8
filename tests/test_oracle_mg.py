"""Pins of the oracle's multigrid layer (no GPU): the paper's stated level sizes,
exact properties of shape-function transfers and Galerkin operators, the
V-cycle as a symmetric positive definite preconditioner, and PCG against a
dense direct solve."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import fem, mg
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "level_sizes.json")


def test_level_sizes_from_paper():
    cases = json.load(open(GOLDEN))["cases"]
    for c in cases:
        nel = tuple(c["nel"])
        for L, dofs in c.get("exact", {}).items():
            got = mg.level_dofs(nel, int(L), ceil=c.get("ceil", False))[-1]
            assert got == dofs, (c["cite"], L, got)
        for limit, L in c.get("limits", {}).items():
            assert mg.plan_levels(nel, 0, int(limit)) == L, (c["cite"], limit)
        if "fine_about" in c:
            fine = mg.level_dofs(nel, 1)[0]
            assert abs(fine - c["fine_about"]) / c["fine_about"] < 0.05


@pytest.mark.parametrize("nel", [(6, 4), (4, 2, 6)])
def test_prolongator_reproduces_linear_fields(nel):
    dim = len(nel)
    P = mg.geometric_prolongator(nel)
    # rows sum to one per component (partition of unity)
    rs = np.asarray(P.sum(axis=1)).ravel()
    assert np.all(rs == 1.0)
    Xf = fem.node_coordinates(nel)
    Xc = fem.node_coordinates([n // 2 for n in nel], 2.0)
    G = np.array([[0.25, -1.0, 0.5], [2.0, 0.125, -0.75], [-0.5, 0.375, 1.5]])[:dim, :dim]
    uc = (Xc @ G.T + 0.5).ravel()
    uf = (Xf @ G.T + 0.5).ravel()
    assert np.max(np.abs(P @ uc - uf)) == 0.0          # dyadic weights: exact
    # rigid-body modes map to rigid-body modes
    assert np.max(np.abs(P @ fem.rigid_body_modes(Xc) - fem.rigid_body_modes(Xf))) == 0.0


@pytest.mark.parametrize("nel", [(8, 6), (4, 4, 6)])
def test_galerkin_is_rediscretisation(nel):
    """Uniform material, no supports: P^T K_h P equals the stiffness matrix of
    the grid with twice the element size (nested spaces).  In 2D KE does not
    depend on h; in 3D KE(2h) = 2 KE(h)."""
    dim = len(nel)
    KE = fem.element_stiffness(dim, 0.3)
    Kh = fem.assemble(nel, np.ones(int(np.prod(nel))), KE)
    cel = tuple(n // 2 for n in nel)
    K2h = fem.assemble(cel, np.ones(int(np.prod(cel))), fem.element_stiffness(dim, 0.3, 2.0))
    Ac = mg.galerkin(mg.geometric_prolongator(nel), Kh)
    assert Ac.nnz == K2h.nnz
    assert np.array_equal(Ac.indptr, K2h.indptr) and np.array_equal(Ac.indices, K2h.indices)
    assert np.max(np.abs(Ac.data - K2h.data)) <= 1e-14 * np.max(np.abs(K2h.data))


def _small_hier(dim=2, nel=(8, 4), L=3, seed=5, omega=0.5, nu=1):
    p = synth.small_case(dim, nel, seed=seed)
    KE = fem.element_stiffness(dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, L, omega=omega, nu_pre=nu, nu_post=nu)
    return p, H


@pytest.mark.parametrize("dim,nel,L", [(2, (16, 8), 4), (3, (8, 4, 4), 3)])
def test_levels_symmetric_spd_and_stencil_pattern(dim, nel, L):
    p, H = _small_hier(dim, nel, L)
    for l, A in enumerate(H.A):
        assert abs(A - A.T).max() <= 1e-14 * abs(A).max()
        assert np.linalg.eigvalsh(A.toarray()).min() > 0
        if l > 0:
            # geometric coarse levels: full block stencil of nodes sharing an element
            cel = tuple(n // 2 ** l for n in nel)
            pat = fem.assemble(cel, np.ones(int(np.prod(cel))), fem.element_stiffness(dim, 0.3))
            assert np.array_equal(A.indptr, pat.indptr) and np.array_equal(A.indices, pat.indices)


def _dense_precond(H):
    n = H.A[0].shape[0]
    return np.column_stack([mg.vcycle(H, e) for e in np.eye(n)])


def test_vcycle_symmetric_positive_definite():
    p, H = _small_hier(2, (8, 4), 3)
    M = _dense_precond(H)
    assert np.max(np.abs(M - M.T)) <= 1e-12 * np.max(np.abs(M))
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


def test_two_grid_contraction():
    """Error propagation I - M A of a two-level cycle contracts in the A norm."""
    p, H = _small_hier(2, (8, 4), 2)
    A = H.A[0].toarray()
    M = _dense_precond(H)
    Lc = np.linalg.cholesky(A)
    Eprop = Lc.T @ (np.eye(A.shape[0]) - M @ A) @ np.linalg.inv(Lc.T)
    assert np.linalg.norm(Eprop, 2) < 1.0


def test_single_level_is_exact():
    p, H = _small_hier(2, (8, 4), 1)
    r = mg.mg_pcg(H, p.loads[0], 1e-12)
    assert r.iters == 1


@pytest.mark.parametrize("uniform", [True, False])
def test_mbb_pcg_matches_dense(uniform):
    p = synth.mbb_2d(uniform)
    KE = fem.element_stiffness(2, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, 3, omega=0.6, nu_pre=2, nu_post=2)
    f = p.loads[0]
    r = mg.mg_pcg(H, f, 1e-13)
    ud = mg.dense_solve(H.A[0], f)
    assert np.linalg.norm(r.u - ud) <= 1e-9 * np.linalg.norm(ud)
    # with a zero start the CG iterate satisfies f.u = u.K u up to ||u|| ||r||
    A0 = H.A[0]
    res = np.linalg.norm(f - A0 @ r.u)
    assert abs(f @ r.u - r.u @ (A0 @ r.u)) <= np.linalg.norm(r.u) * res * 1.01 + 1e-15
    assert r.u[p.fixed].max() == 0.0 and r.u[p.fixed].min() == 0.0


def test_rtol_1e8_compliance_close_to_exact():
    p = synth.mbb_2d(False)
    KE = fem.element_stiffness(2, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, 3, omega=0.6, nu_pre=2, nu_post=2)
    ud = mg.dense_solve(H.A[0], p.loads[0])
    r = mg.mg_pcg(H, p.loads[0], 1e-8)
    assert r.converged and r.relres <= 1e-8
    c_ref = p.loads[0] @ ud
    assert abs(r.compliance - c_ref) <= 1e-9 * abs(c_ref)


# ------------------------------------------------------------- Chebyshev smoothing
def test_chebyshev_residual_polynomial():
    """On A = diag(lam), D = I, b = 1, x0 = 0 the residual after nu steps is the
    scaled Chebyshev polynomial T_nu((theta - lam)/delta) / T_nu(theta/delta)."""
    from numpy.polynomial import chebyshev as C
    lam = np.linspace(0.05, 2.2, 40)
    A = sp.diags(lam).tocsr()
    I = sp.identity(40, format="csr")
    b = np.ones(40)
    theta, delta = 1.2, 0.9
    for nu in (1, 2, 3, 5):
        x = mg.chebyshev_smooth(A, I, b, np.zeros(40), theta, delta, nu)
        Tn = np.zeros(nu + 1)
        Tn[nu] = 1.0
        expect = C.chebval((theta - lam) / delta, Tn) / C.chebval(theta / delta, Tn)
        np.testing.assert_allclose(b - A @ x, expect, rtol=1e-12, atol=1e-14)


def test_power_estimate_converges_to_lmax():
    lam = np.array([1, 2, 3, 4, 5, 6, 7, 8, 9, 20.0])
    A = sp.diags(lam).tocsr()
    est = mg.power_lmax(A, sp.identity(10, format="csr"))
    assert est <= 20.0 + 1e-12 and est >= 20.0 * (1 - 1e-6)
    # start vector values lie in [1, 2) and follow the published hash
    v = mg.power_start(5)
    assert np.all((v >= 1.0) & (v < 2.0))
    assert mg._fmix32(np.array([0]))[0] == 0 and mg._fmix32(np.array([1]))[0] == 0x514E28B7


@pytest.mark.parametrize("nu", [2, 3])
def test_chebyshev_vcycle_spd_and_mbb(nu):
    """The Chebyshev-smoothed V-cycle is a symmetric positive definite
    preconditioner and MG-PCG with it reaches the dense solution."""
    import synth
    p = synth.mbb_2d(False)
    KE = fem.element_stiffness(2, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, 3, nu_pre=nu, nu_post=nu, smoother="chebyshev")
    assert all(c is not None for c in H.cheb[:-1])
    n = H.A[0].shape[0]
    m = fem.free_mask(n, p.fixed)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((n, 6)) * m[:, None]
    V = np.column_stack([mg.vcycle(H, X[:, k]) for k in range(6)])
    G = X.T @ V
    assert np.max(np.abs(G - G.T)) <= 1e-10 * np.max(np.abs(G))
    assert np.all(np.linalg.eigvalsh(0.5 * (G + G.T)) > 0)
    ud = mg.dense_solve(H.A[0], p.loads[0])
    r = mg.mg_pcg(H, p.loads[0], 1e-10)
    assert r.converged
    assert np.linalg.norm(r.u - ud) <= 1e-8 * np.linalg.norm(ud)


def test_block_diag_inverse_hand_built():
    """Point-block inverse on a matrix whose blocks are inverted by hand: the
    off-diagonal blocks are ignored, a non-symmetric block catches a transposed
    fill, and each stored block times A's diagonal block is the identity."""
    A = np.zeros((8, 8))
    A[0:3, 0:3] = [[4, 1, 0], [1, 3, 1], [0, 1, 2]]        # det 18 (cofactor expansion)
    A[3:6, 3:6] = np.diag([2.0, 5.0, 0.5])
    A[0, 3] = A[3, 0] = 7.0                                 # coupling between blocks 0 and 1
    A[2, 5] = A[5, 2] = -3.0
    A = sp.csr_matrix(A[:6, :6])
    D = mg.block_diag_inverse(A, 3).toarray()
    inv0 = np.array([[5, -2, 1], [-2, 8, -4], [1, -4, 11]]) / 18.0   # adjugate / det
    np.testing.assert_allclose(D[0:3, 0:3], inv0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(D[3:6, 3:6], np.diag([0.5, 0.2, 2.0]), rtol=0, atol=1e-15)
    assert np.all(D[0:3, 3:6] == 0) and np.all(D[3:6, 0:3] == 0)
    for b in range(2):
        s = slice(3 * b, 3 * b + 3)
        np.testing.assert_allclose(D[s, s] @ A.toarray()[s, s], np.eye(3), atol=1e-14)
    # a non-symmetric 2x2 block: [[1, 2], [0, 1]]^-1 = [[1, -2], [0, 1]]
    B = sp.csr_matrix(np.array([[1.0, 2.0, 9.0, 0.0], [0.0, 1.0, 0.0, 0.0],
                                [9.0, 0.0, 4.0, 0.0], [0.0, 0.0, 0.0, 8.0]]))
    DB = mg.block_diag_inverse(B, 2).toarray()
    np.testing.assert_array_equal(DB[0:2, 0:2], [[1.0, -2.0], [0.0, 1.0]])
    np.testing.assert_array_equal(DB[2:4, 2:4], [[0.25, 0.0], [0.0, 0.125]])
    assert np.all(DB[0:2, 2:4] == 0)


@pytest.mark.parametrize("nel,rows", [((14, 10), 37), ((6, 4, 6), 100)])
def test_blocked_galerkin_equals_one_shot(nel, rows):
    """P^T A P summed over row blocks has the one-shot pattern and values (to the
    rounding of the re-associated sums)."""
    p = synth.small_case(len(nel), nel, seed=42)
    KE = fem.element_stiffness(p.dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    A = fem.apply_dirichlet(fem.assemble(p.nel, E, KE), p.fixed)
    P = mg.geometric_prolongator(p.nel, p.fixed)
    G1 = mg.galerkin(P, A)
    G2 = mg.galerkin(P, A, block_rows=rows)
    assert np.array_equal(G1.indptr, G2.indptr) and np.array_equal(G1.indices, G2.indices)
    assert np.max(np.abs(G1.data - G2.data)) <= 1e-14 * np.max(np.abs(G1.data))
    H1 = mg.build_geometric(p.nel, E, KE, p.fixed, 3)
    H2 = mg.build_geometric(p.nel, E, KE, p.fixed, 3, lean=True)
    for a, b in zip(H1.A, H2.A):
        assert np.array_equal(a.indices, b.indices)
        assert np.max(np.abs(a.data - b.data)) <= 1e-14 * np.max(np.abs(a.data))
