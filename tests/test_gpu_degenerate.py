"""Degenerate inputs of the solve, against the oracle's sparse direct solve of
its assembled K~ (Sec. 2 supports, Sec. 3.1 stop test): the smallest meshes
that still coarsen (one coarse element per axis, odd counts), uniform solid and
uniform void densities, and loads that vanish after the supports are applied
(zero, or only on supported dofs), which stop before the first iteration with
u = 0.  u is compared at the parity bar of the solve tests (1e-7)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

import synth
from oracle import fem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dense_u(p, rho, f):
    KE = fem.element_stiffness(p.dim, p.nu)
    K = fem.apply_dirichlet(fem.assemble(p.nel, fem.simp(rho, p.p, p.E0, p.Emin), KE), p.fixed).tocsc()
    g = f.copy()
    g[p.fixed] = 0.0
    return spl.spsolve(K, g)


def _gpu(p, rho, L, **kw):
    from paper_2001_01655_amd import Hierarchy
    return Hierarchy(p.nel, rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=L, **kw)


@pytest.mark.parametrize("dim,nel", [(2, (2, 2)), (2, (3, 3)), (2, (5, 2)), (3, (2, 2, 2)), (3, (3, 2, 3))])
@pytest.mark.parametrize("vfp", [32, 64])
def test_smallest_meshes(dim, nel, vfp):
    """Two levels whose coarse level has one or two elements per axis."""
    print(f"smallest mesh {nel} vfp={vfp}", flush=True)
    p = synth.small_case(dim, nel, seed=51, n_rhs=1)
    G = _gpu(p, p.rho, 2, vcycle_fp=vfp, outer=0 if vfp == 32 else 1)
    r = G.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-10)
    G.close()
    ud = _dense_u(p, p.rho, p.loads[0])
    u = r.u.cpu().numpy()
    assert r.converged
    assert np.linalg.norm(u - ud) <= 1e-7 * np.linalg.norm(ud)
    assert np.all(u[p.fixed] == 0.0)


@pytest.mark.parametrize("fill", [1.0, 1e-3])
def test_uniform_density(fill):
    """Uniform solid, and uniform void (E = Emin + (E0 - Emin) 1e-9 everywhere:
    the same operator scaled down, so u scales up by about 5e8)."""
    print(f"uniform density {fill}", flush=True)
    p = synth.small_case(3, (12, 8, 8), seed=52, n_rhs=1)
    rho = np.full_like(p.rho, fill)
    G = _gpu(p, rho, 3, smoother=2, nu_pre=2, nu_post=2)
    r = G.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-10)
    G.close()
    ud = _dense_u(p, rho, p.loads[0])
    assert r.converged
    assert np.linalg.norm(r.u.cpu().numpy() - ud) <= 1e-7 * np.linalg.norm(ud)


@pytest.mark.parametrize("where", ["zero", "supports_only"])
def test_vanishing_load(where):
    """M f = 0: the stop test holds before the first iteration; u = 0 exactly,
    compliance 0 and the reported relative residual 0 (no 0/0)."""
    print(f"vanishing load {where}", flush=True)
    p = synth.small_case(2, (16, 8), seed=53, n_rhs=1)
    f = np.zeros(p.n_dof)
    if where == "supports_only":
        f[p.fixed] = 1.0
    G = _gpu(p, p.rho, 3)
    r = G.solve(torch.tensor(f, device="cuda"), rtol=1e-8)
    G.close()
    assert r.converged
    assert r.iters == [0]
    assert torch.count_nonzero(r.u).item() == 0
    assert r.compliance == [0.0] and r.relres == [0.0]
