"""GPU parity of the geometric-multigrid path against the CPU oracle.

Every case runs through the C ABI (libtopomg.so) on the same seeded inputs as
the oracle.  Sizes span several 256-thread workgroups with ragged tails."""
import numpy as np
import pytest

import synth
from oracle import fem, mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _oracle(p, L, omega=0.5, nu=1, point=False):
    KE = fem.element_stiffness(p.dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, L, omega=omega, nu_pre=nu, nu_post=nu,
                           point_jacobi=point)
    return H, E, KE


def _gpu(p, L, **kw):
    from paper_2001_01655_amd import Hierarchy
    return Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=L, **kw)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# the last two coarsen odd element counts to ceil(n/2) (Sec. 4.3)
CASES = [(2, (28, 12), 3), (3, (10, 6, 4), 2), (3, (12, 8, 8), 3), (2, (13, 7), 3), (3, (9, 5, 7), 3)]


@pytest.mark.parametrize("dim,nel,L", CASES)
def test_fine_apply(dim, nel, L):
    _say(f"fine apply {nel}")
    p = synth.small_case(dim, nel, seed=21)
    H, E, KE = _oracle(p, L)
    G = _gpu(p, L)
    x = np.random.default_rng(3).standard_normal(p.n_dof)
    ref = H.A[0] @ x
    y64 = G.apply(0, torch.tensor(x, device="cuda"), fp=64).cpu().numpy()
    assert _rel(y64, ref) <= 1e-13
    y32 = G.apply(0, torch.tensor(x, device="cuda", dtype=torch.float32), fp=32).cpu().numpy()
    ref32 = H.A[0] @ x.astype(np.float32).astype(np.float64)
    assert _rel(y32, ref32) <= 2e-6
    G.close()


# stencil_kernel 1 runs the large-level coarse operator kernel on these small
# levels too (0 picks by size, which here is always the small-level form)
KERNELS = pytest.mark.parametrize("kern", [0, 1], ids=["by_size", "large_kernel"])


@pytest.mark.parametrize("dim,nel,L", CASES)
@KERNELS
def test_levels_prolongators_dinv(dim, nel, L, kern):
    _say(f"levels {nel} stencil_kernel={kern}")
    p = synth.small_case(dim, nel, seed=22)
    H, E, KE = _oracle(p, L)
    G = _gpu(p, L, stencil_kernel=kern)
    assert G.num_levels() == L
    for l in range(1, L):
        rp, ci, v = G.export_csr(l)
        A = H.A[l]
        assert np.array_equal(rp, A.indptr) and np.array_equal(ci, A.indices), f"pattern level {l}"
        assert _rel(v, A.data) <= 1e-12, f"values level {l}"
        x = np.random.default_rng(l).standard_normal(A.shape[0])
        y = G.apply(l, torch.tensor(x, device="cuda"), fp=64).cpu().numpy()
        assert _rel(y, A @ x) <= 1e-13
    for l in range(L - 1):
        rp, ci, v = G.export_prolongator(l)
        P = H.P[l]
        assert np.array_equal(rp, P.indptr) and np.array_equal(ci, P.indices), f"P pattern {l}"
        assert np.array_equal(v, P.data)
    for l in range(L):
        d = G.export_dinv(l)
        bs = H.bs[l]
        ref = H.Dinv[l].toarray().reshape(-1, bs, H.A[l].shape[0] // bs, bs)
        ref = np.stack([ref[i, :, i, :] for i in range(ref.shape[0])])
        assert _rel(d, ref) <= 1e-11, f"dinv level {l}"
    G.close()


@pytest.mark.parametrize("dim,nel,L", CASES)
@KERNELS
def test_vcycle_fp64(dim, nel, L, kern):
    _say(f"vcycle {nel} stencil_kernel={kern}")
    p = synth.small_case(dim, nel, seed=23)
    H, E, KE = _oracle(p, L)
    G = _gpu(p, L, vcycle_fp=64, stencil_kernel=kern)
    b = H.A[0] @ np.random.default_rng(5).standard_normal(p.n_dof)
    b[p.fixed] = 0.0                      # the V-cycle acts on masked vectors
    ref = mg.vcycle(H, b)
    assert np.all(ref[p.fixed] == 0.0)
    z = G.vcycle(torch.tensor(b, device="cuda"), fp=64).cpu().numpy()
    # the coarsest solve multiplies by an explicit inverse: error ~ cond(A_c) eps
    assert _rel(z, ref) <= 1e-9
    z32 = G.vcycle(torch.tensor(b, device="cuda", dtype=torch.float32), fp=32).cpu().numpy()
    assert _rel(z32, ref) <= 1e-3
    G.close()


@pytest.mark.parametrize("uniform", [True, False])
@pytest.mark.parametrize("vfp,outer", [(64, 1), (32, 0)])
def test_mbb_solve_vs_dense(uniform, vfp, outer):
    """The paper-style MBB half-beam (60x20, 3 levels, omega 0.6, 2/2 sweeps):
    GPU solve at rtol 1e-8 against the exact (dense Cholesky) solution."""
    _say(f"mbb uniform={uniform} vfp={vfp}")
    p = synth.mbb_2d(uniform)
    KE = fem.element_stiffness(2, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    A0 = fem.apply_dirichlet(fem.assemble(p.nel, E, KE), p.fixed)
    ud = mg.dense_solve(A0, p.loads[0])
    G = _gpu(p, 3, omega=0.6, nu_pre=2, nu_post=2, vcycle_fp=vfp, outer=outer)
    r = G.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-8)
    u = r.u.cpu().numpy()
    assert r.converged and r.relres[0] <= 1.2e-8
    assert np.linalg.norm(u - ud) <= 1e-7 * np.linalg.norm(ud)
    c = p.loads[0] @ ud
    assert abs(r.compliance[0] - c) <= 1e-9 * abs(c)
    assert np.all(u[p.fixed] == 0.0)
    G.close()


@pytest.mark.parametrize("dim,nel,L", [(2, (64, 32), 4), (3, (16, 8, 8), 3), (2, (45, 23), 4), (3, (11, 6, 5), 3)])
@pytest.mark.parametrize("vfp", [64, 32])
def test_solve_vs_oracle(dim, nel, L, vfp):
    """u at rtol 1e-8 against the oracle at rtol 1e-12 (contrast 1e9 in E)."""
    _say(f"solve {nel} vfp={vfp}")
    p = synth.small_case(dim, nel, seed=24, n_rhs=2)
    H, E, KE = _oracle(p, L)
    G = _gpu(p, L, vcycle_fp=vfp, outer=0 if vfp == 32 else 1)
    F = torch.tensor(p.loads, device="cuda")
    r = G.solve(F, rtol=1e-8)
    U = r.u.cpu().numpy()
    for k in range(p.loads.shape[0]):
        ref = mg.mg_pcg(H, p.loads[k], 1e-12)
        assert r.converged and r.relres[k] <= 1.2e-8
        e = np.linalg.norm(U[k] - ref.u) / np.linalg.norm(ref.u)
        ce = abs(r.compliance[k] - ref.compliance) / abs(ref.compliance)
        _say(f"  rhs {k}: iters={r.iters[k]} (oracle {ref.iters}) err_u={e:.2e} err_c={ce:.2e}")
        assert e <= 1e-7 and ce <= 1e-9
    G.close()


def test_warm_start_and_update():
    p = synth.small_case(3, (16, 8, 8), seed=25)
    G = _gpu(p, 3)
    f = torch.tensor(p.loads[0], device="cuda")
    r1 = G.solve(f, rtol=1e-8)
    rho2 = synth.density_update(p.rho, p.nel, seed=25, step=1)
    G.update_density(torch.tensor(rho2, device="cuda"))
    r_cold = G.solve(f, rtol=1e-8)
    r_warm = G.solve(f, rtol=1e-8, u0=r1.u)
    assert r_warm.converged and r_cold.converged
    assert r_warm.iters[0] <= r_cold.iters[0]
    diff = (r_warm.u - r_cold.u).norm() / r_cold.u.norm()
    assert float(diff) < 1e-6
    G.close()


@pytest.mark.parametrize("dim,nel,L", [c for c in CASES if c[0] == 3])
def test_vcycle_fp32_matrix_cores(dim, nel, L):
    """The FP32 fine operator on the matrix cores gives the V-cycle of the
    oracle to FP32 accuracy, and agrees with the vector-FMA operator."""
    _say(f"vcycle matrix cores {nel}")
    p = synth.small_case(dim, nel, seed=26)
    H, E, KE = _oracle(p, L)
    b = H.A[0] @ np.random.default_rng(7).standard_normal(p.n_dof)
    b[p.fixed] = 0.0
    ref = mg.vcycle(H, b)
    z = {}
    for mf in (0, 1):
        G = _gpu(p, L, vcycle_fp=32, fine_mfma=mf)
        z[mf] = G.vcycle(torch.tensor(b, device="cuda", dtype=torch.float32), fp=32).cpu().numpy()
        G.close()
    assert _rel(z[1], ref) <= 1e-3
    assert _rel(z[1], z[0]) <= 1e-4


def test_solve_matrix_cores_vs_oracle():
    """Mixed-precision solve with the matrix-core fine operator: u and
    compliance at rtol 1e-8 against the oracle at rtol 1e-12."""
    _say("solve matrix cores (16, 8, 8)")
    p = synth.small_case(3, (16, 8, 8), seed=27, n_rhs=2)
    H, E, KE = _oracle(p, 3)
    G = _gpu(p, 3, vcycle_fp=32, outer=0, fine_mfma=1)
    r = G.solve(torch.tensor(p.loads, device="cuda"), rtol=1e-8)
    U = r.u.cpu().numpy()
    for k in range(p.loads.shape[0]):
        ref = mg.mg_pcg(H, p.loads[k], 1e-12)
        assert r.converged and r.relres[k] <= 1.2e-8
        assert np.linalg.norm(U[k] - ref.u) <= 1e-7 * np.linalg.norm(ref.u)
        assert abs(r.compliance[k] - ref.compliance) <= 1e-9 * abs(ref.compliance)
    G.close()


@pytest.mark.parametrize("dim,nel,L", CASES)
@pytest.mark.parametrize("nu", [2, 3])
@KERNELS
def test_vcycle_chebyshev(dim, nel, L, nu, kern):
    """Chebyshev smoothing (interval from a 12-step power estimate per level):
    the V-cycle in FP64 and FP32 against the oracle's."""
    _say(f"vcycle chebyshev {nel} nu={nu} stencil_kernel={kern}")
    p = synth.small_case(dim, nel, seed=28)
    KE = fem.element_stiffness(p.dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, L, nu_pre=nu, nu_post=nu, smoother="chebyshev")
    b = H.A[0] @ np.random.default_rng(9).standard_normal(p.n_dof)
    b[p.fixed] = 0.0
    ref = mg.vcycle(H, b)
    G = _gpu(p, L, nu_pre=nu, nu_post=nu, smoother=2, vcycle_fp=64, stencil_kernel=kern)
    z = G.vcycle(torch.tensor(b, device="cuda"), fp=64).cpu().numpy()
    assert _rel(z, ref) <= 1e-9
    z32 = G.vcycle(torch.tensor(b, device="cuda", dtype=torch.float32), fp=32).cpu().numpy()
    assert _rel(z32, ref) <= 1e-3
    G.close()


@pytest.mark.parametrize("vfp,outer", [(64, 1), (32, 0)])
def test_solve_chebyshev_vs_oracle(vfp, outer):
    _say(f"solve chebyshev vfp={vfp}")
    p = synth.small_case(3, (16, 8, 8), seed=29, n_rhs=2)
    KE = fem.element_stiffness(3, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, 3, nu_pre=2, nu_post=2, smoother="chebyshev")
    G = _gpu(p, 3, nu_pre=2, nu_post=2, smoother=2, vcycle_fp=vfp, outer=outer)
    r = G.solve(torch.tensor(p.loads, device="cuda"), rtol=1e-8)
    U = r.u.cpu().numpy()
    for k in range(p.loads.shape[0]):
        ref = mg.mg_pcg(H, p.loads[k], 1e-12)
        assert r.converged and r.relres[k] <= 1.2e-8
        assert np.linalg.norm(U[k] - ref.u) <= 1e-7 * np.linalg.norm(ref.u)
        assert abs(r.compliance[k] - ref.compliance) <= 1e-9 * abs(ref.compliance)
        _say(f"  rhs {k}: iters={r.iters[k]} (oracle PCG {ref.iters} at rtol 1e-12)")
    G.close()


@pytest.mark.parametrize("dim,nel,L", CASES)
def test_chebyshev_keeps_block_inverses(dim, nel, L):
    """With Chebyshev smoothing each level's block inverse is stored divided
    by its interval centre; the export undoes that and gives the same blocks
    as the Jacobi hierarchy of the same problem."""
    _say(f"chebyshev dinv {nel}")
    p = synth.small_case(dim, nel, seed=30)
    Gj = _gpu(p, L)
    Gc = _gpu(p, L, smoother=2, nu_pre=2, nu_post=2)
    for l in range(L):
        dj, dc = Gj.export_dinv(l), Gc.export_dinv(l)
        assert _rel(dc, dj) <= 1e-14, f"level {l}"
    Gj.close()
    Gc.close()


def test_update_without_waiting_reports_device_checks_at_the_next_solve():
    """A density update of a geometric hierarchy enqueues its work and returns;
    what the device finds (here a density outside [0, 1]) is reported by the
    next solve, and a good update afterwards solves normally."""
    from paper_2001_01655_amd import TmError
    from paper_2001_01655_amd import _lib as L
    p = synth.small_case(3, (12, 8, 8), seed=31)
    G = _gpu(p, 3)
    f = torch.tensor(p.loads[0], device="cuda")
    bad = p.rho.copy()
    bad[5] = 2.0
    G.update_density(torch.tensor(bad, device="cuda"))
    with pytest.raises(TmError) as e:
        G.solve(f, rtol=1e-8)
    assert e.value.status == L.TM_ERR_ARG
    G.update_density(torch.tensor(p.rho, device="cuda"))
    r = G.solve(f, rtol=1e-8)
    assert r.converged
    H, E, KE = _oracle(p, 3)
    ref = mg.mg_pcg(H, p.loads[0], 1e-12)
    assert np.linalg.norm(r.u.cpu().numpy() - ref.u) <= 1e-7 * np.linalg.norm(ref.u)
    G.close()
