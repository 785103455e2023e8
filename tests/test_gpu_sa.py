"""GPU parity of the smoothed-aggregation levels (hybrid hierarchy) against
the CPU oracle: bit-exact aggregates and sparsity patterns, FP values within
tolerance, and the full solve."""
import numpy as np
import pytest

import synth
from oracle import fem, mg, sa

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (problem, n_geometric, max_coarse): 3D thin-strut lattice and a 2D smoothed field
CASES = [
    ("bridge", (32, 16, 16), 2, 1000),
    ("bridge", (32, 16, 16), 3, 300),
    ("small2d", (64, 32), 2, 300),
    # aggregation below odd-count coarsenings (rigid-body modes at the true node positions)
    ("small2d", (45, 23), 2, 300),
    ("small2d", (45, 27), 3, 100),
    ("small3d", (13, 9, 7), 2, 300),
]


def _problem(kind, nel):
    if kind == "bridge":
        return synth.bridge_3d(nel=nel)
    return synth.small_case(len(nel), nel, seed=31)


def _pair(kind, nel, ngeo, maxc, vfp=64):
    p = _problem(kind, nel)
    KE = fem.element_stiffness(p.dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = sa.build_hybrid(p.nel, E, KE, p.fixed, ngeo, max_coarse=maxc)
    from paper_2001_01655_amd import Hierarchy
    G = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_geometric=ngeo,
                  max_coarse=maxc, vcycle_fp=vfp, outer=1 if vfp == 64 else 0)
    return p, H, G


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("kind,nel,ngeo,maxc", CASES)
def test_aggregation_levels(kind, nel, ngeo, maxc):
    print(f"sa levels {kind} {nel}", flush=True)
    p, H, G = _pair(kind, nel, ngeo, maxc)
    assert "sa" in H.kinds
    assert G.num_levels() == H.L
    for l in range(H.L):
        info = G.level_info(l)
        assert info["n_rows"] == H.A[l].shape[0]
    for l in range(ngeo - 1, H.L - 1):
        agg = G.export_aggregates(l)
        assert np.array_equal(agg, H.aggregates[l]), f"aggregates level {l}"
        rp, ci, v = G.export_prolongator(l)
        P = H.P[l]
        assert np.array_equal(rp, P.indptr) and np.array_equal(ci, P.indices), f"P pattern level {l}"
        assert _rel(v, P.data) <= 1e-10, f"P values level {l}"
    for l in range(ngeo, H.L):
        rp, ci, v = G.export_csr(l)
        A = H.A[l]
        assert np.array_equal(rp, A.indptr) and np.array_equal(ci, A.indices), f"A pattern level {l}"
        assert _rel(v, A.data) <= 1e-10, f"A values level {l}"
    G.close()


@pytest.mark.parametrize("kind,nel,ngeo,maxc", CASES)
def test_aggregation_vcycle_and_solve(kind, nel, ngeo, maxc):
    print(f"sa solve {kind} {nel}", flush=True)
    p, H, G = _pair(kind, nel, ngeo, maxc)
    b = H.A[0] @ np.random.default_rng(7).standard_normal(p.n_dof)
    b[p.fixed] = 0.0
    z = G.vcycle(torch.tensor(b, device="cuda"), fp=64).cpu().numpy()
    assert _rel(z, mg.vcycle(H, b)) <= 1e-8
    f = p.loads[0]
    ref = mg.mg_pcg(H, f, 1e-12)
    for vfp in (64, 32):
        if vfp == 32:
            G.close()
            p, H, G = _pair(kind, nel, ngeo, maxc, vfp=32)
        r = G.solve(torch.tensor(f, device="cuda"), rtol=1e-8)
        u = r.u.cpu().numpy()
        e = np.linalg.norm(u - ref.u) / np.linalg.norm(ref.u)
        ce = abs(r.compliance[0] - ref.compliance) / abs(ref.compliance)
        print(f"  vfp={vfp} iters={r.iters[0]} (oracle {ref.iters} at 1e-12) err_u={e:.2e} err_c={ce:.2e}",
              flush=True)
        assert r.converged and r.relres[0] <= 1.2e-8
        assert e <= 1e-7 and ce <= 1e-9
    G.close()


def test_aggregation_update_rebuilds_levels():
    p = synth.bridge_3d(nel=(32, 16, 16))
    from paper_2001_01655_amd import Hierarchy
    G = Hierarchy(p.nel, p.rho, p.fixed, n_geometric=2, max_coarse=1000)
    f = torch.tensor(p.loads[0], device="cuda")
    r1 = G.solve(f, rtol=1e-8)
    rho2 = np.where(p.rho > 0.5, 1.0, 0.2)
    G.update_density(torch.tensor(rho2, device="cuda"))
    r2 = G.solve(f, rtol=1e-8)
    KE = fem.element_stiffness(3, 0.3)
    H = sa.build_hybrid(p.nel, fem.simp(rho2, 3, 1, 1e-9), KE, p.fixed, 2, max_coarse=1000)
    assert np.array_equal(G.export_aggregates(1), H.aggregates[1])
    ref = mg.mg_pcg(H, p.loads[0], 1e-12)
    assert r1.converged and r2.converged
    assert np.linalg.norm(r2.u.cpu().numpy() - ref.u) <= 1e-7 * np.linalg.norm(ref.u)
    G.close()


@pytest.mark.parametrize("kind,nel,ngeo,maxc", CASES[:2])
def test_aggregation_vcycle_chebyshev(kind, nel, ngeo, maxc):
    """Chebyshev smoothing on every level of the hybrid hierarchy (aggregation
    levels included): the FP64 V-cycle against the oracle's."""
    print(f"sa chebyshev {kind} {nel}", flush=True)
    p = _problem(kind, nel)
    KE = fem.element_stiffness(p.dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = sa.build_hybrid(p.nel, E, KE, p.fixed, ngeo, max_coarse=maxc, nu_pre=2, nu_post=2,
                        smoother="chebyshev")
    from paper_2001_01655_amd import Hierarchy
    G = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_geometric=ngeo,
                  max_coarse=maxc, vcycle_fp=64, outer=1, nu_pre=2, nu_post=2, smoother=2)
    b = H.A[0] @ np.random.default_rng(11).standard_normal(p.n_dof)
    b[p.fixed] = 0.0
    z = G.vcycle(torch.tensor(b, device="cuda"), fp=64).cpu().numpy()
    assert _rel(z, mg.vcycle(H, b)) <= 1e-8
    G.close()


def test_hybrid_updates_reuse_memory_and_match_fresh_setup():
    """Density updates of a hybrid hierarchy rebuild its aggregation levels in
    grow-only arenas: once the sizes have been seen, further updates take no
    device memory, and each solve equals, bit for bit, the solve of a
    hierarchy set up from scratch for the same densities."""
    from paper_2001_01655_amd import Hierarchy
    print("hybrid updates", flush=True)
    p = synth.small_case(3, (16, 12, 8), seed=81)
    opts = dict(p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_geometric=2, max_coarse=300)
    f = torch.tensor(p.loads[0], device="cuda")
    G = Hierarchy(p.nel, p.rho, p.fixed, **opts)
    rhos = [synth.density_update(p.rho, p.nel, seed=81, step=t) for t in range(1, 5)]
    held = []
    for t, rho in enumerate(rhos):
        G.update_density(torch.tensor(rho, device="cuda"))
        r = G.solve(f, rtol=1e-8)
        torch.cuda.synchronize()
        held.append(torch.cuda.memory_allocated())
        F = Hierarchy(p.nel, rho, p.fixed, **opts)
        rf = F.solve(f, rtol=1e-8)
        assert r.converged and r.iters == rf.iters, f"update {t}"
        assert torch.equal(r.u, rf.u), f"update {t}"
        F.close()
        del rf
        torch.cuda.synchronize()
        held[-1] = torch.cuda.memory_allocated()
    print(f"  bytes held after each update: {held}", flush=True)
    assert held[2] == held[1] and held[3] == held[2]
    G.close()


@pytest.mark.parametrize("kind,nel,ngeo,maxc", [CASES[1], CASES[2], CASES[5]])
def test_setup_without_lds_staging_is_bitwise_equal(kind, nel, ngeo, maxc):
    """Option sa_lds = 1 takes the paths that long rows and large aggregates
    take (every Galerkin product block by block, Gram-Schmidt in device
    memory, one prolongator block per group): every aggregation level's
    prolongator and operator, and the solve, are bitwise those of the default."""
    from paper_2001_01655_amd import Hierarchy
    print(f"sa without lds {kind} {nel}", flush=True)
    p = _problem(kind, nel)
    Gs = [Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_geometric=ngeo,
                    max_coarse=maxc, sa_lds=m) for m in (0, 1)]
    L = Gs[0].num_levels()
    assert Gs[1].num_levels() == L
    for l in range(ngeo - 1, L - 1):
        for a, b in zip(Gs[0].export_prolongator(l), Gs[1].export_prolongator(l)):
            assert np.array_equal(a, b), f"prolongator level {l}"
    for l in range(ngeo, L):
        for a, b in zip(Gs[0].export_csr(l), Gs[1].export_csr(l)):
            assert np.array_equal(a, b), f"operator level {l}"
    f = torch.tensor(p.loads[0], device="cuda")
    r0, r1 = (G.solve(f, rtol=1e-8) for G in Gs)
    assert r0.iters == r1.iters and torch.equal(r0.u, r1.u)
    for G in Gs:
        G.close()
