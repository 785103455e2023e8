"""Pins of the oracle's finite-element layer against facts fixed by geometry,
by mechanics and by closed-form integration (no GPU)."""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import fem
import synth


# ---------------------------------------------------------------- numbering
@pytest.mark.parametrize("nel", [(3, 2), (4, 3, 2)])
def test_connectivity_by_coordinates(nel):
    """Element corners found by coordinate lookup; orientation checked
    geometrically (2D counter-clockwise from the lower-left corner; 3D bottom
    face counter-clockwise, top face directly above)."""
    dim = len(nel)
    ids = {}
    for idx, c in enumerate(itertools.product(*[range(n + 1) for n in reversed(nel)])):
        ids[tuple(reversed(c))] = idx            # x varies fastest
    conn = fem.connectivity(nel)
    coords = {v: k for k, v in ids.items()}
    for e, row in enumerate(conn):
        pts = np.array([coords[n] for n in row], dtype=float)
        lo = pts.min(axis=0)
        assert tuple(pts[0]) == tuple(lo)                      # first = lower corner
        assert np.all(pts.max(axis=0) - lo == 1)               # unit cell
        quad = pts[:4, :2]
        area = 0.5 * sum(quad[i, 0] * quad[(i + 1) % 4, 1] - quad[(i + 1) % 4, 0] * quad[i, 1]
                         for i in range(4))
        assert area == pytest.approx(1.0)                      # counter-clockwise
        if dim == 3:
            assert np.all(pts[:4, 2] == lo[2])
            assert np.all(pts[4:] - pts[:4] == np.array([0, 0, 1]))
        # element id: x fastest
        assert e == int(lo[0] + nel[0] * (lo[1] + (nel[1] * lo[2] if dim == 3 else 0)))


# ---------------------------------------------------------------- KE
def _ke_closed_form(dim, nu, h, E=1.0):
    """KE from the Lame form of isotropic elasticity,
    a(u,v) = lam div u div v + 2 mu eps(u):eps(v), with the tensor-product 1D
    integrals of linear hat functions done by hand:
      int phi_s phi_t = h/3 (s=t) or h/6;  int phi_s' phi_t = sgn(s)/2;
      int phi_s' phi_t' = sgn(s) sgn(t)/h.
    2D is plane stress (lam* = E nu / (1 - nu^2)), unit thickness."""
    mu = E / (2 * (1 + nu))
    lam = E * nu / (1 - nu * nu) if dim == 2 else E * nu / ((1 + nu) * (1 - 2 * nu))
    loc = fem.LOCAL_2D if dim == 2 else fem.LOCAL_3D
    sg = lambda s: 1.0 if s else -1.0
    M = lambda s, t: h / 3 if s == t else h / 6

    def A(c, d, a, b):      # int d_c N_a d_d N_b
        v = 1.0
        for k in range(dim):
            sa, sb = loc[a][k], loc[b][k]
            if k == c and k == d:
                v *= sg(sa) * sg(sb) / h
            elif k == c:
                v *= sg(sa) / 2
            elif k == d:
                v *= sg(sb) / 2
            else:
                v *= M(sa, sb)
        return v

    n = 2 ** dim
    K = np.zeros((dim * n, dim * n))
    for a, b, c, d in itertools.product(range(n), range(n), range(dim), range(dim)):
        v = lam * A(c, d, a, b) + mu * A(d, c, a, b)
        if c == d:
            v += mu * sum(A(k, k, a, b) for k in range(dim))
        K[dim * a + c, dim * b + d] = v
    return K


@pytest.mark.parametrize("dim,nu,h", [(2, 0.3, 1.0), (2, 0.45, 2.0), (3, 0.3, 1.0), (3, 0.2, 0.5)])
def test_ke_closed_form(dim, nu, h):
    KE = fem.element_stiffness(dim, nu, h)
    ref = _ke_closed_form(dim, nu, h)
    assert np.max(np.abs(KE - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("dim", [2, 3])
def test_ke_spectrum_and_rigid_modes(dim):
    KE = fem.element_stiffness(dim, 0.3)
    assert np.array_equal(KE, KE.T)
    coords = (fem.LOCAL_2D if dim == 2 else fem.LOCAL_3D).astype(float)
    B = fem.rigid_body_modes(coords)
    assert np.max(np.abs(KE @ B)) < 1e-13
    ev = np.linalg.eigvalsh(KE)
    nz = 3 if dim == 2 else 6
    assert np.all(np.abs(ev[:nz]) < 1e-13)
    assert ev[nz] > 1e-3
    # row sums per component vanish (translations)
    assert np.max(np.abs(KE.reshape(-1, 2 ** dim, dim).sum(axis=1))) < 1e-13


def test_ke_scaling_with_h():
    assert np.allclose(fem.element_stiffness(2, 0.3, 3.0), fem.element_stiffness(2, 0.3, 1.0), rtol=0, atol=1e-14)
    assert np.allclose(fem.element_stiffness(3, 0.3, 2.0), 2 * fem.element_stiffness(3, 0.3, 1.0), rtol=0, atol=1e-14)


def test_simp_endpoints():
    r = np.array([0.0, 1.0, 0.5])
    E = fem.simp(r, 3.0, 1.0, 1e-9)
    assert E[0] == 1e-9 and E[1] == 1.0
    assert E[2] == pytest.approx(1e-9 + (1 - 1e-9) * 0.125)


# ---------------------------------------------------------------- assembly
@pytest.mark.parametrize("nel", [(5, 3), (3, 2, 2)])
def test_assembly_pattern_symmetry_nullspace(nel):
    dim = len(nel)
    KE = fem.element_stiffness(dim, 0.3)
    rng = np.random.default_rng(0)
    E = rng.uniform(0.1, 1.0, size=int(np.prod(nel)))
    K = fem.assemble(nel, E, KE)
    assert (abs(K - K.T)).max() <= 1e-15 * abs(K).max()
    # structural pattern: node pairs sharing an element, counted by brute force
    conn = fem.connectivity(nel)
    pairs = set()
    for row in conn:
        for a in row:
            for b in row:
                pairs.add((a, b))
    assert K.nnz == len(pairs) * dim * dim
    B = fem.rigid_body_modes(fem.node_coordinates(nel))
    assert np.max(np.abs(K @ B)) < 1e-12 * np.max(np.abs(B))


@pytest.mark.parametrize("nel", [(6, 4), (4, 3, 3)])
def test_patch_test(nel):
    """Uniform material, linear displacement prescribed on the boundary: the
    interior solution is the same linear field."""
    dim = len(nel)
    K = fem.assemble(nel, np.ones(int(np.prod(nel))), fem.element_stiffness(dim, 0.3))
    X = fem.node_coordinates(nel)
    G = np.array([[0.3, -0.2, 0.1], [0.05, 0.4, -0.3], [0.2, 0.1, -0.1]])[:dim, :dim]
    u = (X @ G.T + np.array([0.7, -0.4, 0.2])[:dim]).ravel()
    on_b = np.any((X == 0) | (X == np.array(nel)[None, :]), axis=1)
    bd = np.repeat(on_b, dim)
    I, Bn = ~bd, bd
    Kc = K.tocsr()
    uI = spla.spsolve(Kc[I][:, I].tocsc(), -(Kc[I][:, Bn] @ u[Bn]))
    assert np.max(np.abs(uI - u[I])) < 1e-12


def test_dirichlet_rows_and_matfree():
    p = synth.small_case(3, (4, 2, 2), seed=3)
    KE = fem.element_stiffness(3, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    Kt = fem.apply_dirichlet(fem.assemble(p.nel, E, KE), p.fixed)
    for d in p.fixed[:5]:
        row = Kt.getrow(d)
        assert row.nnz == 1 and row.indices[0] == d and row.data[0] == 1.0
    x = np.random.default_rng(1).standard_normal(p.n_dof)
    y1 = Kt @ x
    y2 = fem.apply_matfree(p.nel, E, KE, p.fixed, x)
    assert np.max(np.abs(y1 - y2)) <= 1e-14 * np.max(np.abs(y1))


def _compliance(nel, rho, fixed, f, p=3.0, E0=1.0, Emin=1e-9, nu=0.3):
    import scipy.sparse.linalg as spla
    KE = fem.element_stiffness(len(nel), nu)
    K = fem.apply_dirichlet(fem.assemble(nel, fem.simp(rho, p, E0, Emin), KE), fixed)
    fm = f * fem.free_mask(len(f), fixed)
    u = spla.spsolve(K.tocsc(), fm)
    return fm @ u, u, KE


@pytest.mark.parametrize("nel", [(6, 4), (3, 2, 2)])
def test_sensitivity_matches_finite_differences(nel):
    """Central differences of c(rho) = f^T K(rho)^-1 f pin the analytic
    sensitivity (Sec. 2) element by element."""
    import synth
    p = synth.small_case(len(nel), nel, seed=31, n_rhs=1)
    rho = 0.3 + 0.6 * np.random.default_rng(4).uniform(size=int(np.prod(nel)))
    c, u, KE = _compliance(nel, rho, p.fixed, p.loads[0])
    dc = fem.compliance_sensitivity(nel, rho, 3.0, 1.0, 1e-9, KE, u)
    h = 1e-6
    for e in range(len(rho)):
        rp, rm = rho.copy(), rho.copy()
        rp[e] += h
        rm[e] -= h
        fd = (_compliance(nel, rp, p.fixed, p.loads[0])[0] - _compliance(nel, rm, p.fixed, p.loads[0])[0]) / (2 * h)
        assert abs(fd - dc[e]) <= 1e-6 * np.max(np.abs(dc)), e


def test_sensitivity_homogeneity():
    """With Emin = 0, K(t rho) = t^p K(rho), so c(t rho) = t^-p c and Euler's
    identity gives sum_e rho_e dc/d rho_e = -p c exactly."""
    import synth
    nel = (8, 4)
    p = synth.small_case(2, nel, seed=32, n_rhs=1)
    rho = 0.2 + 0.8 * np.random.default_rng(5).uniform(size=32)
    c, u, KE = _compliance(nel, rho, p.fixed, p.loads[0], p=3.0, Emin=0.0)
    dc = fem.compliance_sensitivity(nel, rho, 3.0, 1.0, 0.0, KE, u)
    assert abs(rho @ dc + 3.0 * c) <= 1e-10 * abs(c)
    assert np.all(dc <= 0.0)


@pytest.mark.parametrize("nel,ppb", [((13, 7), 3), ((5, 4, 6), 2), ((6, 3, 4), 8)])
def test_blocked_assembly_equals_one_shot(nel, ppb):
    """The slab-by-slab K~ is the one-shot assemble + apply_dirichlet: the same
    pattern, and each entry the sum of the same (at most 2^dim) element terms,
    up to the order in which the sparse conversion adds them."""
    p = synth.small_case(len(nel), nel, seed=41)
    KE = fem.element_stiffness(p.dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    A = fem.apply_dirichlet(fem.assemble(p.nel, E, KE), p.fixed)
    B = fem.assemble_dirichlet_blocked(p.nel, E, KE, p.fixed, planes_per_block=ppb)
    assert np.array_equal(A.indptr, B.indptr) and np.array_equal(A.indices, B.indices)
    absK = fem.assemble(p.nel, E, np.abs(KE))          # bound on each entry's terms
    bound = 8 * np.finfo(float).eps * np.abs(fem.apply_dirichlet(absK, p.fixed).data)
    assert np.all(np.abs(A.data - B.data) <= bound)
