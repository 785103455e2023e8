"""Pins of the oracle's smoothed-aggregation layer (no GPU)."""
import itertools
from collections import deque

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, mg, sa
import synth

M32 = 0xFFFFFFFF


def test_fmix32_inverts_with_published_constants():
    """MurmurHash3's 32-bit finaliser is a bijection; undo it with the inverses
    of its published multipliers (0x85ebca6b, 0xc2b2ae35)."""
    inv1 = pow(0x85EBCA6B, -1, 1 << 32)
    inv2 = pow(0xC2B2AE35, -1, 1 << 32)

    def unshift(h, s):
        x = h
        for _ in range(32 // s + 1):
            x = h ^ (x >> s)
        return x & M32

    rng = np.random.default_rng(0)
    for i in list(range(50)) + [int(v) for v in rng.integers(0, 1 << 32, size=200)]:
        h = sa.fmix32(i)
        x = unshift(h, 16)
        x = (x * inv2) & M32
        x = unshift(x, 13)
        x = (x * inv1) & M32
        x = unshift(x, 16)
        assert x == i
    assert sa.fmix32(0) == 0


# ---------------------------------------------------------------- strength
def _strength_bruteforce(A, bs, beta):
    D = A.toarray()
    n = D.shape[0] // bs
    blk = lambda i, j: D[i * bs:(i + 1) * bs, j * bs:(j + 1) * bs]
    S = np.zeros((n, n), bool)
    for i in range(n):
        for j in range(n):
            if i != j and np.any(blk(i, j) != 0):
                S[i, j] = np.linalg.norm(blk(i, j)) ** 2 > beta * np.linalg.norm(blk(i, i)) * np.linalg.norm(blk(j, j))
    return S | S.T


def test_strength_matches_pairwise_definition():
    p = synth.small_case(2, (6, 4), seed=2)
    A = fem.assemble(p.nel, fem.simp(p.rho, 3, 1, 1e-9), fem.element_stiffness(2, 0.3))
    S = sa.strength(A, 2, 0.003).toarray() > 0
    assert np.array_equal(S, _strength_bruteforce(A, 2, 0.003))


def test_strength_uniform_material():
    """2D: every stencil neighbour is strong.  3D: face and edge neighbours
    are strong, the eight body-diagonal neighbours are weak."""
    K2 = fem.assemble((4, 4), np.ones(16), fem.element_stiffness(2, 0.3))
    S2 = sa.strength(K2, 2)
    P2 = (fem.assemble((4, 4), np.ones(16), np.ones((8, 8))) != 0).astype(float).tobsr((2, 2))
    assert S2.nnz == P2.nnz // 4 - 25     # all off-diagonal node pairs
    nel = (4, 4, 4)
    K3 = fem.assemble(nel, np.ones(64), fem.element_stiffness(3, 0.3))
    S3 = sa.strength(K3, 3)
    X = fem.node_coordinates(nel).astype(int)
    c = fem.node_index(nel, np.array([[2, 2, 2]]))[0]
    strong = set(S3.indices[S3.indptr[c]:S3.indptr[c + 1]])
    for off in itertools.product([-1, 0, 1], repeat=3):
        if off == (0, 0, 0):
            continue
        j = fem.node_index(nel, np.array([[2 + off[0], 2 + off[1], 2 + off[2]]]))[0]
        assert (j in strong) == (np.count_nonzero(off) < 3), off


def test_strength_cuts_stiffness_jumps():
    """The coupling from an interface node into the soft side is kept for mild
    contrast and cut once the soft side is about an order of magnitude softer
    or more (Sec. 4, remark after the strength formula)."""
    nel = (8, 4)
    ex = np.tile(np.arange(8), 4)

    def couples(c):
        E = np.where(ex < 4, 1.0, c)
        A = fem.assemble(nel, E, fem.element_stiffness(2, 0.3))
        S = sa.strength(A, 2).toarray() > 0
        i = fem.node_index(nel, np.array([[4, 2]]))[0]      # on the interface
        j = fem.node_index(nel, np.array([[5, 2]]))[0]      # one element into the soft side
        return S[i, j]

    assert couples(1.0) and couples(0.5)
    assert not couples(1e-2) and not couples(1e-9)


# ---------------------------------------------------------------- aggregation
def _lfmis2_aggregates_bruteforce(S):
    """Roots: scan nodes by key, admit a node iff no admitted root lies within
    graph distance 2.  Then root neighbours; then the remaining nodes join the
    pass-1 neighbour whose root has the smallest key."""
    n = S.shape[0]
    adj = [set(S.indices[S.indptr[i]:S.indptr[i + 1]]) for i in range(n)]
    dist = np.full((n, n), 99)
    for s in range(n):
        dist[s, s] = 0
        q = deque([s])
        while q:
            u = q.popleft()
            for v in adj[u]:
                if dist[s, v] > dist[s, u] + 1:
                    dist[s, v] = dist[s, u] + 1
                    q.append(v)
    key = [(sa.fmix32(i), i) for i in range(n)]
    roots = []
    for u in sorted(range(n), key=lambda i: key[i]):
        if all(dist[u, r] > 2 for r in roots):
            roots.append(u)
    roots.sort()
    agg = {r: g for g, r in enumerate(roots)}
    root_of = {r: r for r in roots}
    for i in range(n):
        if i not in root_of:
            rs = [r for r in roots if dist[i, r] == 1]
            if rs:
                root_of[i] = rs[0]
    first = dict(root_of)
    for i in range(n):
        if i not in first:
            cands = [first[j] for j in adj[i] if j in first]
            root_of[i] = min(cands, key=lambda r: key[r])
    return np.array([agg[root_of[i]] for i in range(n)]), set(roots), dist


@pytest.mark.parametrize("seed", range(6))
def test_aggregation_matches_bruteforce(seed):
    rng = np.random.default_rng(seed)
    n = 40
    M = np.triu(rng.random((n, n)) < 0.08, 1)
    M = M | M.T
    S = sp.csr_matrix(M.astype(float))
    agg, is_root, n_agg = sa.aggregate(S)
    ref, roots, dist = _lfmis2_aggregates_bruteforce(S)
    assert np.array_equal(agg, ref)
    assert set(np.nonzero(is_root)[0]) == roots
    R = sorted(roots)
    for a, b in itertools.combinations(R, 2):
        assert dist[a, b] >= 3
    assert all(min(dist[i, r] for r in R) <= 2 for i in range(n))
    assert n_agg == len(R)


def test_aggregation_invariants_on_strength_graph():
    p = synth.bridge_3d(nel=(16, 8, 8))
    A = mg.build_geometric(p.nel, fem.simp(p.rho, 3, 1, 1e-9), fem.element_stiffness(3, 0.3),
                           p.fixed, 2).A[1]
    S = sa.strength(A, 3)
    agg, is_root, n_agg = sa.aggregate(S)
    assert agg.min() == 0 and agg.max() == n_agg - 1
    assert np.array_equal(np.sort(agg[is_root]), np.arange(n_agg))   # ids by root order
    assert np.all(np.diff(np.nonzero(is_root)[0]) > 0)


# ---------------------------------------------------------------- T and P
def _setup_level(nel=(16, 8, 8), n_geo=2):
    p = synth.bridge_3d(nel=nel)
    H = mg.build_geometric(p.nel, fem.simp(p.rho, 3, 1, 1e-9), fem.element_stiffness(3, 0.3),
                           p.fixed, n_geo)
    A = H.A[-1]
    lev = [n // 2 ** (n_geo - 1) for n in nel]
    B = fem.rigid_body_modes(fem.node_coordinates(lev, 2.0 ** (n_geo - 1)))
    return A, B


def test_tentative_prolongator():
    A, B = _setup_level()
    S = sa.strength(A, 3)
    agg, _, n_agg = sa.aggregate(S)
    T, Bc = sa.tentative(agg, n_agg, B, 3)
    assert np.max(np.abs(T @ Bc - B)) <= 1e-12 * np.max(np.abs(B))
    TT = (T.T @ T).toarray()
    d = np.diag(TT)
    assert set(np.round(d, 12)) <= {0.0, 1.0}
    live = d > 0.5
    assert np.max(np.abs(TT[np.ix_(live, live)] - np.eye(live.sum()))) < 1e-12
    sizes = np.bincount(agg, minlength=n_agg)
    for g in np.nonzero(sizes == 1)[0]:                     # 3 dofs cannot carry 6 modes
        assert np.sum(d[6 * g:6 * g + 6] > 0.5) == 3
    # R factor upper triangular with non-negative diagonal
    for g in range(n_agg):
        R = Bc[6 * g:6 * g + 6]
        assert np.allclose(np.tril(R, -1), 0) and np.all(np.diag(R) >= 0)


def test_smoothed_prolongator_pattern_and_weight():
    A, B = _setup_level()
    agg, _, n_agg = sa.aggregate(sa.strength(A, 3))
    T, _ = sa.tentative(agg, n_agg, B, 3)
    P = sa.smoothed_prolongator(A, T, 3)
    pat = ((abs(T) + abs(mg._ones(A) @ mg._ones(T))) > 0).astype(float).tocsr()
    pat.sort_indices()
    assert np.array_equal(P.indptr, pat.indptr) and np.array_equal(P.indices, pat.indices)
    Dinv = mg.block_diag_inverse(A, 3)
    lam = np.abs(np.linalg.eigvals((Dinv @ A).toarray())).max()
    w = sa.jacobi_weight(A, Dinv)
    assert w * lam <= 4.0 / 3.0 + 1e-12                  # inf-norm bounds the spectral radius


def test_hybrid_solve_matches_direct():
    p = synth.bridge_3d(nel=(16, 8, 8))
    E = fem.simp(p.rho, 3, 1, 1e-9)
    KE = fem.element_stiffness(3, 0.3)
    H = sa.build_hybrid(p.nel, E, KE, p.fixed, 2, max_coarse=300)
    assert H.kinds[0] == "geo" and "sa" in H.kinds
    for A in H.A[1:]:
        assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
        assert np.linalg.eigvalsh(A.toarray()).min() > 0
    r = mg.mg_pcg(H, p.loads[0], 1e-12)
    ud = mg.dense_solve(H.A[0], p.loads[0])
    assert np.linalg.norm(r.u - ud) <= 1e-6 * np.linalg.norm(ud)
    assert abs(r.compliance - p.loads[0] @ ud) <= 1e-10 * abs(p.loads[0] @ ud)


def test_jacobi_weight_hand_computed():
    """omega = (4/3) / ||D^-1 A||_inf on a 4x4 matrix with 2x2 point blocks,
    D^-1 A and its row sums worked out by hand:
      block 0 = [[4, 1], [1, 2]], inverse [[2, -1], [-1, 4]] / 7;
      block 1 = diag(3, 4), inverse diag(1/3, 1/4);
      D^-1 A rows: [7, 0, 4, 2]/7, [0, 7, -2, -8]/7, [2/3, 0, 1, 0], [0, -1/2, 0, 1];
      absolute row sums 13/7, 17/7, 5/3, 3/2, so omega = (4/3)(7/17) = 28/51.
    Point Jacobi (diag A) would give rows summing to 7/4, 5/2, 5/3, 3/2 and
    omega 8/15; a halved weight 14/51."""
    A = sp.csr_matrix(np.array([[4.0, 1.0, 2.0, 0.0],
                                [1.0, 2.0, 0.0, -2.0],
                                [2.0, 0.0, 3.0, 0.0],
                                [0.0, -2.0, 0.0, 4.0]]))
    Dinv = mg.block_diag_inverse(A, 2)
    DA = np.array([[1.0, 0.0, 4 / 7, 2 / 7],
                   [0.0, 1.0, -2 / 7, -8 / 7],
                   [2 / 3, 0.0, 1.0, 0.0],
                   [0.0, -0.5, 0.0, 1.0]])
    np.testing.assert_allclose((Dinv @ A).toarray(), DA, rtol=0, atol=1e-15)
    w = sa.jacobi_weight(A, Dinv)
    assert abs(w - 28.0 / 51.0) <= 1e-15
    # the weight is fixed by the block inverse: point Jacobi gives another value
    assert abs(sa.jacobi_weight(A, mg.point_diag_inverse(A)) - 8.0 / 15.0) <= 1e-15
