"""Pins of the ceil(n/2) geometric coarsening (Sec. 4.3) in the oracle: the
per-axis interpolation, the Galerkin operator on an odd grid against direct
assembly on the (non-uniform) coarse mesh, and a solve through such levels
against a dense solve."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import fem, mg


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 8, 13])
def test_axis_interpolation(n):
    W = mg.axis_prolongator(n).toarray()
    nc = mg.coarse_count(n)
    assert W.shape == (n + 1, nc + 1)
    assert np.allclose(W.sum(axis=1), 1.0, rtol=0, atol=0)              # partition of unity
    pos = np.minimum(2 * np.arange(nc + 1), n)
    assert np.array_equal(W @ pos.astype(float), np.arange(n + 1, dtype=float))   # linear fields
    if n % 2 == 0:                                                        # even: w(i - 2I)
        ref = np.zeros_like(W)
        for i in range(n + 1):
            for I in range(nc + 1):
                d = abs(i - 2 * I)
                ref[i, I] = 1.0 if d == 0 else (0.5 if d == 1 else 0.0)
        assert np.array_equal(W, ref)


def _assemble_box(cnel, sizes_per_axis, nu):
    """K on a tensor mesh whose element (X, Y[, Z]) has edge lengths
    (sx[X], sy[Y][, sz[Z]])."""
    dim = len(cnel)
    ed = fem.element_dofs(cnel)
    n = dim * int(np.prod([c + 1 for c in cnel]))
    rows, cols, vals = [], [], []
    for e, idx in enumerate(np.ndindex(*cnel[::-1])):                     # slowest axis first
        ijk = idx[::-1]
        KE = fem.element_stiffness_box(dim, nu, [sizes_per_axis[a][ijk[a]] for a in range(dim)])
        rows.append(np.repeat(ed[e], ed.shape[1]))
        cols.append(np.tile(ed[e], ed.shape[1]))
        vals.append(KE.ravel())
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    return K.tocsr()


@pytest.mark.parametrize("nel", [(5, 3), (7, 4), (5, 3, 3), (4, 5, 3)])
def test_galerkin_on_odd_grid_is_the_coarse_mesh_operator(nel):
    dim, nu = len(nel), 0.3
    Kh = fem.assemble(nel, np.ones(int(np.prod(nel))), fem.element_stiffness(dim, nu))
    P = mg.geometric_prolongator(nel)
    KH = (P.T @ Kh @ P).toarray()
    cnel = [mg.coarse_count(n) for n in nel]
    sizes = []
    for n, c in zip(nel, cnel):
        pos = np.minimum(2 * np.arange(c + 1), n)
        sizes.append(np.diff(pos).astype(float))
    ref = _assemble_box(cnel, sizes, nu).toarray()
    assert np.allclose(KH, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("dim,nel,L", [(2, (13, 7), 3), (3, (9, 5, 7), 3), (3, (11, 6, 5), 3)])
def test_odd_hierarchy_solves(dim, nel, L):
    p = synth.small_case(dim, nel, seed=61)
    KE = fem.element_stiffness(dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, L)
    sizes = [A.shape[0] for A in H.A]
    assert sizes == mg.level_dofs(nel, L, ceil=True)
    for A in H.A:
        assert abs(A - A.T).max() <= 1e-12 * abs(A).max()
        assert np.linalg.eigvalsh(A.toarray()).min() > 0
    A0 = fem.apply_dirichlet(fem.assemble(p.nel, E, KE), p.fixed)
    f = p.loads[0].copy()
    f[p.fixed] = 0.0
    ud = mg.dense_solve(A0, f)
    r = mg.mg_pcg(H, p.loads[0], 1e-10)
    assert np.linalg.norm(r.u - ud) <= 1e-8 * np.linalg.norm(ud)


@pytest.mark.parametrize("nel,levels,h", [((13, 7), 3, 1.0), ((9, 5, 7), 3, 0.5), ((33, 17), 4, 2.0)])
def test_level_node_positions_closed_form(nel, levels, h):
    """Composing 'coarse node I sits on fine node min(2I, n)' over l levels
    places node I of level l at h * min(2^l I, n_0)."""
    from oracle import sa
    cur, pos = sa.level_node_positions(nel, levels, h)
    sc = 2 ** (levels - 1)
    for n0, m, p in zip(nel, cur, pos):
        assert len(p) == m + 1
        assert np.array_equal(p, h * np.minimum(sc * np.arange(m + 1), n0).astype(float))
        assert p[-1] == h * n0                     # the last node stays on the boundary


@pytest.mark.parametrize("dim,nel,ngeo,maxc", [(2, (45, 23), 2, 300), (2, (45, 27), 3, 100), (3, (13, 9, 7), 2, 300)])
def test_hybrid_below_odd_coarsening(dim, nel, ngeo, maxc):
    """Aggregation on a level reached through odd counts: the tentative
    prolongator reproduces the rigid-body modes at the level's true node
    positions, every level is SPD, and PCG matches a dense solve."""
    from oracle import sa
    p = synth.small_case(dim, nel, seed=62)
    KE = fem.element_stiffness(dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = sa.build_hybrid(p.nel, E, KE, p.fixed, ngeo, max_coarse=maxc)
    assert H.kinds[ngeo - 1:] and all(k == "sa" for k in H.kinds[ngeo - 1:])
    for A in H.A:
        assert np.linalg.eigvalsh(A.toarray()).min() > 0
    cur, pos = sa.level_node_positions(p.nel, ngeo, p.h)
    grids = np.meshgrid(*[pos[d] for d in reversed(range(dim))], indexing="ij")
    coords = np.stack([g.ravel() for g in reversed(grids)], axis=1)
    B = fem.rigid_body_modes(coords)
    T, Bc = sa.tentative(H.aggregates[ngeo - 1], H.P[ngeo - 1].shape[1] // B.shape[1], B, dim)
    assert np.allclose(T @ Bc, B, atol=1e-12 * np.abs(B).max())
    A0 = fem.apply_dirichlet(fem.assemble(p.nel, E, KE), p.fixed)
    f = p.loads[0].copy()
    f[p.fixed] = 0.0
    ud = mg.dense_solve(A0, f)
    r = mg.mg_pcg(H, p.loads[0], 1e-10)
    assert np.linalg.norm(r.u - ud) <= 1e-8 * np.linalg.norm(ud)
