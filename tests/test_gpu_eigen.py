"""Stability eigenproblem on the GPU (Sec. 2 stress stiffness, Algorithm 2
generalized Davidson) against the oracle: the stress-stiffness operator on
seeded displacement fields (odd and ragged grids, the E_sigma cutoff, both
dimensions), the Davidson eigenvalues and vectors with FP64 and FP32
preconditioning, forced restarts, the iteration limit, the error paths, and
the 256 x 1024 column at full size (sampled rows, properties)."""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import buckling, davidson, fem, mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _hier(p, levels, **kw):
    from paper_2001_01655_amd import Hierarchy
    return Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=levels, **kw)


def _seeded(n, k, seed):
    return np.random.default_rng(seed).standard_normal((k, n)) if k > 1 else \
        np.random.default_rng(seed).standard_normal(n)


@pytest.mark.parametrize("case", [("2d", (13, 7), 0.1), ("3d", (5, 4, 3), 0.1), ("2d", (16, 8), 0.0),
                                  ("3d", (6, 6, 4), 1.0)])
def test_stress_stiffness_apply_vs_oracle(case):
    dim_s, nel, rho_min = case
    dim = len(nel)
    print(f"stress stiffness {nel} rho_min={rho_min}", flush=True)
    p = synth.small_case(dim, nel, seed=23)
    H = _hier(p, 2)
    u = _seeded(p.n_dof, 1, 5)
    x = _seeded(p.n_dof, 1, 6)
    H.stress_stiffness(torch.tensor(u, device="cuda"), rho_min=rho_min)
    y = H.apply_stress_stiffness(torch.tensor(x, device="cuda")).cpu().numpy()
    Ks = buckling.stress_stiffness(p.nel, u, p.rho, p.p, p.E0, p.nu, p.fixed, rho_min=rho_min)
    ref = Ks @ x
    bound = 64 * np.finfo(float).eps * (abs(Ks) @ np.abs(x))
    assert np.all(np.abs(y - ref) <= bound + 1e-300)
    # symmetric as an operator on the device
    x2 = _seeded(p.n_dof, 1, 7)
    y2 = H.apply_stress_stiffness(torch.tensor(x2, device="cuda")).cpu().numpy()
    assert abs(x2 @ y - x @ y2) <= 1e-12 * (np.abs(x2) @ (abs(Ks) @ np.abs(x)))
    H.close()


def _oracle_problem(p, levels):
    KE = fem.element_stiffness(p.dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    Ho = mg.build_geometric(p.nel, E, KE, p.fixed, levels)
    K = Ho.A[0]
    u = mg.dense_solve(K, p.loads[0])
    Ks = buckling.stress_stiffness(p.nel, u, p.rho, p.p, p.E0, p.nu, p.fixed)
    return Ho, K, Ks


def _start(n, k, fixed, seed):
    V0 = np.random.default_rng(seed).standard_normal((n, k))
    V0[fixed] = 0.0
    return V0


@pytest.mark.parametrize("case,fp", [("column", 64), ("small3d", 64), ("column", 32), ("odd2d", 64)])
def test_eigs_vs_oracle(case, fp):
    if case == "column":
        p, levels = synth.column_2d(nel=(8, 32), seed=2), 3
    elif case == "odd2d":
        p, levels = synth.small_case(2, (13, 9), seed=8), 3
    else:
        p, levels = synth.small_case(3, (4, 4, 6), seed=5), 2
    print(f"eigs {case} fp{fp}", flush=True)
    Ho, K, Ks = _oracle_problem(p, levels)
    V0 = _start(K.shape[0], 10, p.fixed, 0)
    ref = davidson.generalized_davidson(lambda v: Ks @ v, lambda v: K @ v, lambda r: mg.vcycle(Ho, r), V0, nev=6)
    H = _hier(p, levels)
    r = H.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-13)
    H.stress_stiffness(r.u)
    lam, Phi, it, nc, st = H.eigs(torch.tensor(V0.T.copy(), device="cuda"), nev=6, precond_fp=fp)
    print(f"  gpu iters {it} oracle {ref.iters}; lambda {lam}", flush=True)
    assert st == 0 and nc == 6
    assert np.allclose(lam, ref.theta, rtol=1e-8, atol=0)
    Pg = Phi.cpu().numpy().T
    assert np.allclose(Pg.T @ (K @ Pg), np.eye(6), atol=1e-9)
    cosang = np.abs(np.sum(Pg * (K @ ref.Phi), axis=0))
    assert np.all(cosang > 1 - 1e-6)
    if fp == 64:
        # same algorithm, same preconditioner up to rounding: the same number of
        # expansions, except where a stagnation test sits at its threshold
        assert abs(it - ref.iters) <= max(2, ref.iters // 10)
    H.close()


def test_eigs_restarts_nev1_and_limits():
    from paper_2001_01655_amd import TmError
    p = synth.column_2d(nel=(8, 32), seed=3)
    Ho, K, Ks = _oracle_problem(p, 3)
    V0 = _start(K.shape[0], 4, p.fixed, 1)
    want = sla.eigh(Ks.toarray()[np.ix_(*(2 * [fem.free_mask(K.shape[0], p.fixed) > 0]))],
                    K.toarray()[np.ix_(*(2 * [fem.free_mask(K.shape[0], p.fixed) > 0]))],
                    eigvals_only=True)[::-1]
    H = _hier(p, 3)
    r = H.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-13)
    H.stress_stiffness(r.u)
    v0 = torch.tensor(V0.T.copy(), device="cuda")
    lam, _, it, nc, st = H.eigs(v0, nev=3, j_min=4, j_max=6, precond_fp=64)
    assert st == 0 and it > 6 and np.allclose(lam, want[:3], rtol=1e-8)
    lam1, _, _, nc1, st1 = H.eigs(v0[:1], nev=1, j_min=2, j_max=5, want_vectors=False)
    assert st1 == 0 and nc1 == 1 and np.isclose(lam1[0], want[0], rtol=1e-8)
    lam2, _, it2, nc2, st2 = H.eigs(v0, nev=3, j_min=4, j_max=6, max_iters=2)
    assert st2 == 1 and it2 == 2 and nc2 < 3
    for bad in [dict(nev=0), dict(nev=10, j_min=10), dict(j_max=33), dict(precond_fp=16), dict(tol=-1.0)]:
        with pytest.raises(TmError) as e:
            H.eigs(v0, **bad)
        assert e.value.status == -1
    dep = torch.stack([v0[0], v0[0]])
    with pytest.raises(TmError) as e:
        H.eigs(dep, nev=1, j_min=3, j_max=5)
    assert e.value.status == -1
    # a density update makes the stress stiffness stale
    H.update_density(torch.tensor(p.rho, device="cuda"))
    with pytest.raises(TmError) as e:
        H.eigs(v0)
    assert e.value.status == -6
    with pytest.raises(TmError) as e:
        H.apply_stress_stiffness(v0[0])
    assert e.value.status == -6
    H.close()


def _patch_row(p, u, node, rho_min=0.1):
    """Oracle rows of node `node` (one per component) from the elements around
    it only: the stress stiffness of the sub-mesh of those elements."""
    nx, ny = p.nel
    i, j = node % (nx + 1), node // (nx + 1)
    x0, x1 = max(0, i - 1), min(nx - 1, i)
    y0, y1 = max(0, j - 1), min(ny - 1, j)
    sub = (x1 - x0 + 1, y1 - y0 + 1)
    ex, ey = np.meshgrid(np.arange(x0, x1 + 1), np.arange(y0, y1 + 1))
    rho = p.rho[(ey * nx + ex).ravel()]
    nxs, nys = np.meshgrid(np.arange(x0, x1 + 2), np.arange(y0, y1 + 2))
    gnodes = (nys * (nx + 1) + nxs).ravel()
    us = np.stack([u[2 * gnodes], u[2 * gnodes + 1]], axis=1).ravel()
    Ks = buckling.stress_stiffness(sub, us, rho, p.p, p.E0, p.nu, np.array([], dtype=np.int64), rho_min=rho_min)
    loc = (j - y0) * (sub[0] + 1) + (i - x0)
    return gnodes, Ks.toarray()[2 * loc:2 * loc + 2]


def test_column_full_size_sampled_rows_and_eigenpairs():
    """The 256 x 1024 column: K_sigma~ x at sampled nodes against the oracle's
    rows from each node's own elements (seeded u and x, the web design), then
    six eigenpairs of the prismatic column with FP32 preconditioning:
    K~-orthonormal, descending, positive, residuals within the stopping tests,
    and the leading one near Euler's load (b = 256, L = 1024)."""
    p = synth.column_2d()
    H = _hier(p, 5)
    u = _seeded(p.n_dof, 1, 11)
    x = _seeded(p.n_dof, 1, 12)
    H.stress_stiffness(torch.tensor(u, device="cuda"))
    y = H.apply_stress_stiffness(torch.tensor(x, device="cuda")).cpu().numpy()
    free = fem.free_mask(p.n_dof, p.fixed)
    xm = free * x
    rng = np.random.default_rng(13)
    nodes = list(rng.integers(0, p.n_nodes, 64)) + [0, p.nel[0], p.n_nodes - 1, (p.nel[0] + 1) * 5]
    for nd in nodes:
        gnodes, rows = _patch_row(p, u, int(nd))
        xs = np.stack([xm[2 * gnodes], xm[2 * gnodes + 1]], axis=1).ravel()
        ref = free[2 * nd:2 * nd + 2] * (rows @ xs)
        bound = 64 * np.finfo(float).eps * (np.abs(rows) @ np.abs(xs)) + 1e-300
        assert np.all(np.abs(y[2 * nd:2 * nd + 2] - ref) <= bound), nd
    H.close()
    # eigenpairs of the prismatic column (the uniform start design of an
    # optimisation; designs with voids need thousands of expansions)
    p = synth.column_2d(uniform=True)
    H = _hier(p, 5)
    r = H.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-8)
    H.stress_stiffness(r.u)
    V0 = torch.tensor(_start(p.n_dof, 10, p.fixed, 3).T.copy(), device="cuda")
    lam, Phi, it, nc, st = H.eigs(V0, nev=6)
    print(f"  column: {it} expansions, lambda {lam}", flush=True)
    assert st == 0 and nc == 6
    assert np.all(np.diff(lam) <= 0) and lam[-1] > 0
    pcr = np.pi ** 2 * (256.0 ** 3 / 12.0) / (4.0 * 1024.0 ** 2)
    # L / b = 4: shear flexibility lowers the load below Euler's by a few percent
    assert 0.0 < lam[0] * pcr - 1.0 < 0.08
    G = torch.empty((6, 6), dtype=torch.float64)
    KP = [H.apply(0, Phi[i]) for i in range(6)]
    for a in range(6):
        for b in range(6):
            G[a, b] = float(Phi[a] @ KP[b])
    assert torch.allclose(G, torch.eye(6, dtype=torch.float64), atol=1e-8)
    for i in range(6):
        res = H.apply_stress_stiffness(Phi[i]) - lam[i] * KP[i]
        rel = float(res.norm()) / (abs(lam[i]) * float(KP[i].norm()))
        print(f"  pair {i}: relative residual {rel:.2e}", flush=True)
        assert rel <= 1e-3
    H.close()


@pytest.mark.parametrize("variant", ["chebyshev", "hybrid", "fp32_3d"])
def test_eigs_other_preconditioners_vs_oracle(variant):
    """Davidson with a Chebyshev-smoothed V-cycle (2/2), with the smoothed-
    aggregation hybrid (2 geometric levels, aggregation below), and with an
    FP32 V-cycle in 3D: the same eigenvalues as the oracle's Davidson with the
    matching oracle preconditioner."""
    from oracle import sa
    print(f"eigs {variant}", flush=True)
    if variant == "chebyshev":
        p, levels = synth.column_2d(nel=(16, 32), seed=4), 3
        kw = dict(smoother=2, nu_pre=2, nu_post=2)
    elif variant == "hybrid":
        p, levels = synth.column_2d(nel=(16, 64), seed=5), None
        kw = dict(n_geometric=2, max_coarse=200)
    else:
        p, levels = synth.small_case(3, (6, 4, 8), seed=9), 2
        kw = {}
    KE = fem.element_stiffness(p.dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    if variant == "chebyshev":
        Ho = mg.build_geometric(p.nel, E, KE, p.fixed, levels, nu_pre=2, nu_post=2, smoother="chebyshev")
    elif variant == "hybrid":
        Ho = sa.build_hybrid(p.nel, E, KE, p.fixed, 2, max_coarse=200)
    else:
        Ho = mg.build_geometric(p.nel, E, KE, p.fixed, levels)
    K = Ho.A[0]
    u = mg.dense_solve(K, p.loads[0])
    Ks = buckling.stress_stiffness(p.nel, u, p.rho, p.p, p.E0, p.nu, p.fixed)
    V0 = _start(K.shape[0], 10, p.fixed, 2)
    ref = davidson.generalized_davidson(lambda v: Ks @ v, lambda v: K @ v, lambda r: mg.vcycle(Ho, r), V0, nev=6)
    assert ref.converged
    if levels is not None:
        kw["n_levels"] = levels
    from paper_2001_01655_amd import Hierarchy
    H = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, **kw)
    if variant == "hybrid":
        assert H.num_levels() == Ho.L
    r = H.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-13)
    H.stress_stiffness(r.u)
    fp = 32 if variant == "fp32_3d" else 64
    lam, Phi, it, nc, st = H.eigs(torch.tensor(V0.T.copy(), device="cuda"), nev=6, precond_fp=fp)
    print(f"  gpu iters {it} oracle {ref.iters}", flush=True)
    assert st == 0 and nc == 6
    assert np.allclose(lam, ref.theta, rtol=1e-8, atol=0)
    Pg = Phi.cpu().numpy().T
    assert np.allclose(Pg.T @ (K @ Pg), np.eye(6), atol=1e-9)
    if fp == 64:
        assert abs(it - ref.iters) <= max(2, ref.iters // 10)
    H.close()


def test_eigs_degenerate_and_largest_space():
    """No stress (u = 0): K_sigma~ = 0, all six eigenvalues 0 without an
    expansion; the largest search space (j_max 32) gives the same eigenvalues
    as the default one."""
    p = synth.column_2d(nel=(8, 32), seed=2)
    H = _hier(p, 3)
    V0 = _start(p.n_dof, 10, p.fixed, 0)
    v0 = torch.tensor(V0.T.copy(), device="cuda")
    H.stress_stiffness(torch.zeros(p.n_dof, dtype=torch.float64, device="cuda"))
    y = H.apply_stress_stiffness(torch.ones(p.n_dof, dtype=torch.float64, device="cuda"))
    assert float(y.abs().max()) == 0.0
    lam, Phi, it, nc, st = H.eigs(v0, nev=6)
    assert st == 0 and it == 0 and nc == 6 and np.all(lam == 0.0)
    r = H.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-13)
    H.stress_stiffness(r.u)
    a, _, ita, nca, sta = H.eigs(v0, nev=6, precond_fp=64)
    b, _, itb, ncb, stb = H.eigs(v0, nev=6, j_min=10, j_max=32, precond_fp=64)
    assert sta == 0 and stb == 0 and np.allclose(a, b, rtol=1e-8)
    print(f"  j_max 25: {ita} expansions, j_max 32: {itb}", flush=True)
    H.close()


def test_eigs_restart_from_previous_eigenvectors():
    """Start vectors = converged eigenvectors (plus seeded ones): the same six
    eigenvalues after far fewer expansions; start vectors given in any scale
    and with entries on supported dofs (ignored) work the same."""
    p = synth.column_2d(nel=(8, 32), seed=2)
    H = _hier(p, 3)
    r = H.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-13)
    H.stress_stiffness(r.u)
    V0 = torch.tensor(_start(p.n_dof, 10, p.fixed, 0).T.copy(), device="cuda")
    lam, Phi, it, nc, st = H.eigs(V0, nev=6, precond_fp=64)
    assert st == 0
    warm = torch.cat([Phi * 3.0, V0[:4]])
    warm[:, torch.tensor(p.fixed, device="cuda")] = 1.0          # ignored by the solver
    lam2, _, it2, nc2, st2 = H.eigs(warm, nev=6, precond_fp=64)
    print(f"  cold {it} expansions, from the eigenvectors {it2}", flush=True)
    assert st2 == 0 and nc2 == 6 and np.allclose(lam2, lam, rtol=1e-8)
    assert it2 <= it // 4
    H.close()


def _patch_rows_nd(p, u, node, rho_min=0.1):
    """Oracle rows (one per component) of `node` from its own elements only, any
    dimension: the stress stiffness of the sub-mesh of those elements."""
    dim, nel = p.dim, p.nel
    nn = [n + 1 for n in nel]
    idx = [node % nn[0], (node // nn[0]) % nn[1]] + ([node // (nn[0] * nn[1])] if dim == 3 else [])
    lo = [max(0, c - 1) for c in idx]
    hi = [min(n - 1, c) for c, n in zip(idx, nel)]
    sub = tuple(h - l + 1 for l, h in zip(lo, hi))
    eg = np.meshgrid(*[np.arange(l, h + 1) for l, h in zip(lo, hi)][::-1], indexing="ij")
    ecoords = [g.ravel() for g in eg[::-1]]
    eid = ecoords[0] + nel[0] * (ecoords[1] + (nel[1] * ecoords[2] if dim == 3 else 0))
    ng = np.meshgrid(*[np.arange(l, h + 2) for l, h in zip(lo, hi)][::-1], indexing="ij")
    ncoords = [g.ravel() for g in ng[::-1]]
    gnodes = ncoords[0] + nn[0] * (ncoords[1] + (nn[1] * ncoords[2] if dim == 3 else 0))
    us = np.stack([u[dim * gnodes + c] for c in range(dim)], axis=1).ravel()
    Ks = buckling.stress_stiffness(sub, us, p.rho[eid], p.p, p.E0, p.nu, np.array([], dtype=np.int64),
                                   rho_min=rho_min)
    sn = [s + 1 for s in sub]
    loc = (idx[0] - lo[0]) + sn[0] * ((idx[1] - lo[1]) + (sn[1] * (idx[2] - lo[2]) if dim == 3 else 0))
    return gnodes, Ks.toarray()[dim * loc:dim * loc + dim]


def test_cantilever3d_full_size_stress_stiffness_and_eigenpairs():
    """192 x 96 x 96 cantilever (5.4M dofs): K_sigma~ x at sampled nodes against
    the oracle's rows from each node's own elements (seeded u and x), then
    Davidson on the real stress state (FP32 V-cycle, at most 300 expansions):
    descending Ritz values, K-orthonormal vectors, converged pairs within the
    stopping tests."""
    p = synth.get("cantilever3d")
    H = _hier(p, 6)
    u = _seeded(p.n_dof, 1, 21)
    x = _seeded(p.n_dof, 1, 22)
    H.stress_stiffness(torch.tensor(u, device="cuda"))
    y = H.apply_stress_stiffness(torch.tensor(x, device="cuda")).cpu().numpy()
    free = fem.free_mask(p.n_dof, p.fixed)
    xm = free * x
    rng = np.random.default_rng(23)
    nodes = list(rng.integers(0, p.n_nodes, 40)) + [0, p.n_nodes - 1, p.nel[0], (p.nel[0] + 1) * (p.nel[1] + 1) * 5 + 7]
    for nd in nodes:
        nd = int(nd)
        gnodes, rows = _patch_rows_nd(p, u, nd)
        xs = np.stack([xm[3 * gnodes + c] for c in range(3)], axis=1).ravel()
        ref = free[3 * nd:3 * nd + 3] * (rows @ xs)
        bound = 64 * np.finfo(float).eps * (np.abs(rows) @ np.abs(xs)) + 1e-300
        assert np.all(np.abs(y[3 * nd:3 * nd + 3] - ref) <= bound), nd
    r = H.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-8)
    H.stress_stiffness(r.u)
    V0 = torch.tensor(_start(p.n_dof, 10, p.fixed, 4).T.copy(), device="cuda")
    lam, Phi, it, nc, st = H.eigs(V0, nev=6, max_iters=300)
    print(f"  cantilever3d: {it} expansions, {nc} converged, lambda {lam}", flush=True)
    assert st in (0, 1) and np.all(np.diff(lam) <= 0)
    KP = [H.apply(0, Phi[i]) for i in range(6)]
    G = np.array([[float(Phi[a] @ KP[b]) for b in range(6)] for a in range(6)])
    assert np.allclose(G, np.eye(6), atol=1e-8)
    for i in range(nc):
        res = H.apply_stress_stiffness(Phi[i]) - lam[i] * KP[i]
        rel = float(res.norm()) / (abs(lam[i]) * float(KP[i].norm()))
        print(f"  pair {i}: relative residual {rel:.2e}", flush=True)
        assert rel <= 1e-3
    H.close()
