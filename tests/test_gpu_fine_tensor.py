"""The 3D fine operator in the tensor-product form (option fine_tensor):
the matrix-free operator K~ = sum_e E_e KE of Sec. 3.1, with KE applied as 45
couplings between per-axis sum / difference modes of an element's corner
values, element columns marched up node planes in 32 x 8 blocks.

Checked through the V-cycle (every smoothing step and residual of the fine
level runs this operator) against the oracle's V-cycle and against the node
gather form, in FP32 and in FP64 (the same code; FP64 pins it to 1e-11 of the
node gather), and through solves against the oracle, on grids that cut the
32 x 8 column tiles and the plane ranges raggedly; n >= 2 fixes the node planes
per workgroup (1 leaves it to the library)."""
import numpy as np
import pytest

import synth
from oracle import fem, mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (nel, levels, fine_tensor)
CASES = [((12, 8, 8), 3, 1), ((17, 31, 9), 3, 1), ((33, 16, 20), 3, 3), ((40, 20, 21), 3, 7),
         ((31, 29, 6), 2, 2), ((16, 15, 15), 3, 16)]


def _gpu(p, L, **kw):
    from paper_2001_01655_amd import Hierarchy
    return Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=L, **kw)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("nel,L,ft", CASES)
@pytest.mark.parametrize("smoother", ["jacobi", "chebyshev"])
def test_vcycle_tensor_form(nel, L, ft, smoother):
    print(f"tensor form vcycle {nel} L={L} fine_tensor={ft} {smoother}", flush=True)
    p = synth.small_case(3, nel, seed=41)
    KE = fem.element_stiffness(3, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    cheb = smoother == "chebyshev"
    nu = 2 if cheb else 1
    H = mg.build_geometric(p.nel, E, KE, p.fixed, L, omega=0.5, nu_pre=nu, nu_post=nu,
                           smoother="chebyshev" if cheb else "jacobi")
    b = H.A[0] @ np.random.default_rng(13).standard_normal(p.n_dof)
    b[p.fixed] = 0.0
    ref = mg.vcycle(H, b)
    z = {}
    for form in (ft, 0):
        G = _gpu(p, L, nu_pre=nu, nu_post=nu, smoother=2 if cheb else 0, vcycle_fp=32, fine_tensor=form)
        z[form] = G.vcycle(torch.tensor(b, device="cuda", dtype=torch.float32), fp=32).cpu().numpy()
        G.close()
    e_ref, e_gather = _rel(z[ft], ref), _rel(z[ft], z[0])
    print(f"  vs oracle {e_ref:.2e}, vs node gather {e_gather:.2e} (gather vs oracle {_rel(z[0], ref):.2e})",
          flush=True)
    # each FP32 form within the FP32 V-cycle's accuracy of the oracle (the
    # two summation orders differ by up to ~1e-4 at the 1e9 stiffness
    # contrast); the same code in FP64 is held to 1e-11 of the FP64 node
    # gather below
    assert e_ref <= 1e-3
    assert e_gather <= 1e-3
    assert np.all(z[ft][p.fixed] == 0.0)


@pytest.mark.parametrize("ft", [1, 5])
def test_solve_tensor_form_vs_oracle(ft):
    """Mixed-precision FCG with the tensor form in its V-cycle: u and
    compliance at rtol 1e-8 against the oracle at rtol 1e-12."""
    print(f"tensor form solve fine_tensor={ft}", flush=True)
    p = synth.small_case(3, (20, 18, 11), seed=42, n_rhs=2)
    KE = fem.element_stiffness(3, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, 3, nu_pre=2, nu_post=2, smoother="chebyshev")
    G = _gpu(p, 3, nu_pre=2, nu_post=2, smoother=2, vcycle_fp=32, outer=0, fine_tensor=ft)
    r = G.solve(torch.tensor(p.loads, device="cuda"), rtol=1e-8)
    U = r.u.cpu().numpy()
    for k in range(p.loads.shape[0]):
        ref = mg.mg_pcg(H, p.loads[k], 1e-12)
        assert r.converged and r.relres[k] <= 1.2e-8
        assert np.linalg.norm(U[k] - ref.u) <= 1e-7 * np.linalg.norm(ref.u)
        assert abs(r.compliance[k] - ref.compliance) <= 1e-9 * abs(ref.compliance)
        print(f"  rhs {k}: iters={r.iters[k]}", flush=True)
    G.close()


@pytest.mark.parametrize("nel,L,ft", CASES[:4])
def test_vcycle_tensor_form_fp64(nel, L, ft):
    """The FP64 form (used by the FP64 V-cycle and by the outer q = K~p with
    its partial sums): the FP64 V-cycle against the oracle's and against the
    FP64 node gather."""
    print(f"tensor form fp64 vcycle {nel} fine_tensor={ft}", flush=True)
    p = synth.small_case(3, nel, seed=43)
    KE = fem.element_stiffness(3, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, L, nu_pre=2, nu_post=2, smoother="chebyshev")
    b = H.A[0] @ np.random.default_rng(14).standard_normal(p.n_dof)
    b[p.fixed] = 0.0
    ref = mg.vcycle(H, b)
    z = {}
    for form in (ft, 0):
        G = _gpu(p, L, nu_pre=2, nu_post=2, smoother=2, vcycle_fp=64, fine_tensor=form)
        z[form] = G.vcycle(torch.tensor(b, device="cuda"), fp=64).cpu().numpy()
        G.close()
    e_ref, e_gather = _rel(z[ft], ref), _rel(z[ft], z[0])
    print(f"  vs oracle {e_ref:.2e}, vs node gather {e_gather:.2e}", flush=True)
    assert e_ref <= 1e-9
    assert e_gather <= 1e-11


def test_solve_fp64_pcg_tensor_form_vs_oracle():
    """FP64 V-cycle in PCG, both fine operators (outer q = K~p with p^T q and
    p^T r, and the V-cycle's) in the FP64 tensor form: u and compliance at rtol
    1e-8 against the oracle at rtol 1e-12."""
    print("tensor form fp64 pcg solve", flush=True)
    p = synth.small_case(3, (20, 18, 11), seed=44, n_rhs=2)
    KE = fem.element_stiffness(3, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, 3, nu_pre=2, nu_post=2, smoother="chebyshev")
    G = _gpu(p, 3, nu_pre=2, nu_post=2, smoother=2, vcycle_fp=64, outer=1, fine_tensor=1)
    r = G.solve(torch.tensor(p.loads, device="cuda"), rtol=1e-8)
    U = r.u.cpu().numpy()
    for k in range(p.loads.shape[0]):
        ref = mg.mg_pcg(H, p.loads[k], 1e-12)
        assert r.converged and r.relres[k] <= 1.2e-8
        assert np.linalg.norm(U[k] - ref.u) <= 1e-7 * np.linalg.norm(ref.u)
        assert abs(r.compliance[k] - ref.compliance) <= 1e-9 * abs(ref.compliance)
        print(f"  rhs {k}: iters={r.iters[k]} (oracle {ref.iters})", flush=True)
    G.close()


# stencil_kernel 3 with even fine element counts: level 1 is applied from the
# fine moduli (2 x 2 x 2 fine elements per level-1 element), supports masked
# per sub-element
L1_CASES = [((12, 8, 8), 3, "clamp"), ((16, 10, 6), 3, "corner"), ((40, 18, 22), 3, "clamp"),
            ((66, 34, 20), 4, "corner")]


@pytest.mark.parametrize("nel,L,support", L1_CASES)
def test_apply_level1_tensor_form(nel, L, support):
    """Level 1 in the tensor form (the Galerkin product P^T M K M P of Sec.
    3.2 applied element by element from the fine moduli, FP32) against the
    oracle's assembled level-1 operator, as the FP32 applies of the other
    levels are held; corner pins mask single sub-elements' corners, the clamp
    a whole face."""
    print(f"level-1 tensor form apply {nel} {support}", flush=True)
    p = synth.small_case(3, nel, seed=45, support=support)
    KE = fem.element_stiffness(3, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, L)
    x = np.random.default_rng(16).standard_normal(H.A[1].shape[0])
    ref32 = H.A[1] @ x.astype(np.float32).astype(np.float64)
    G = _gpu(p, L, stencil_kernel=3)
    y32 = G.apply(1, torch.tensor(x, device="cuda", dtype=torch.float32), fp=32).cpu().numpy()
    G.close()
    e = _rel(y32, ref32)
    print(f"  vs oracle {e:.2e}", flush=True)
    assert e <= 2e-6


@pytest.mark.parametrize("nel,L,support", L1_CASES)
@pytest.mark.parametrize("smoother", ["jacobi", "chebyshev"])
def test_vcycle_level1_tensor_form(nel, L, support, smoother):
    """The FP32 V-cycle with level 1 in the tensor form against the oracle's
    V-cycle and against the stored level-1 stencil.  Pinned at four corners the
    problem is nearly singular and no FP32 V-cycle follows the FP64 oracle to
    1e-3 (the stored stencil's is ~2e-2 off): there the form must be as close
    to the oracle as the stored stencil and agree with it to FP32 rounding."""
    print(f"level-1 tensor form {nel} L={L} {support} {smoother}", flush=True)
    p = synth.small_case(3, nel, seed=45, support=support)
    KE = fem.element_stiffness(3, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    cheb = smoother == "chebyshev"
    nu = 2 if cheb else 1
    H = mg.build_geometric(p.nel, E, KE, p.fixed, L, omega=0.5, nu_pre=nu, nu_post=nu,
                           smoother="chebyshev" if cheb else "jacobi")
    b = H.A[0] @ np.random.default_rng(15).standard_normal(p.n_dof)
    b[p.fixed] = 0.0
    ref = mg.vcycle(H, b)
    z = {}
    for kern in (3, 1):       # 3: level 1 in the tensor form; 1: stored stencils on every level
        G = _gpu(p, L, nu_pre=nu, nu_post=nu, smoother=2 if cheb else 0, vcycle_fp=32, stencil_kernel=kern)
        z[kern] = G.vcycle(torch.tensor(b, device="cuda", dtype=torch.float32), fp=32).cpu().numpy()
        G.close()
    e_ref, e_st, e_st_ref = _rel(z[3], ref), _rel(z[3], z[1]), _rel(z[1], ref)
    print(f"  vs oracle {e_ref:.2e}, vs stored stencil {e_st:.2e} (stored vs oracle {e_st_ref:.2e})", flush=True)
    if support == "clamp":
        assert e_ref <= 1e-3
        assert e_st <= 1e-3
    else:
        assert e_ref <= 1.5 * e_st_ref + 1e-3
        assert e_st <= 1e-2


def test_solve_level1_tensor_form_vs_oracle():
    """Mixed-precision FCG with level 1 in the tensor form, two load cases
    (one launch for both): u and compliance against the oracle."""
    print("level-1 tensor form solve", flush=True)
    p = synth.small_case(3, (24, 14, 12), seed=46, n_rhs=2)
    KE = fem.element_stiffness(3, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, 3, nu_pre=2, nu_post=2, smoother="chebyshev")
    G = _gpu(p, 3, nu_pre=2, nu_post=2, smoother=2, vcycle_fp=32, outer=0, stencil_kernel=3)
    r = G.solve(torch.tensor(p.loads, device="cuda"), rtol=1e-8)
    U = r.u.cpu().numpy()
    for k in range(p.loads.shape[0]):
        ref = mg.mg_pcg(H, p.loads[k], 1e-12)
        assert r.converged and r.relres[k] <= 1.2e-8
        assert np.linalg.norm(U[k] - ref.u) <= 1e-7 * np.linalg.norm(ref.u)
        assert abs(r.compliance[k] - ref.compliance) <= 1e-9 * abs(ref.compliance)
        print(f"  rhs {k}: iters={r.iters[k]} (oracle {ref.iters})", flush=True)
    G.close()
