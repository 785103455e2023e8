"""The caller's allocator of tm_setup (tm_allocator): a hierarchy fed by
torch's caching allocator gives the same solution as one on hipMalloc, its
device memory is visible to torch while it lives and returned when it is
destroyed, and the admission estimate tm_plan_bytes covers what a hierarchy
and its solve states actually take."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu(p, L, **kw):
    from paper_2001_01655_amd import Hierarchy
    return Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=L, **kw)


@pytest.mark.parametrize("opts", [{}, dict(smoother=2, nu_pre=2, nu_post=2)], ids=["jacobi", "chebyshev"])
def test_torch_allocator_solve_equals_hipmalloc_solve(opts):
    print(f"allocator solve {opts}", flush=True)
    p = synth.small_case(3, (20, 12, 10), seed=61, n_rhs=2)
    F = torch.tensor(p.loads, device="cuda")
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    Gt = _gpu(p, 3, allocator="torch", **opts)
    held = torch.cuda.memory_allocated() - base
    assert held >= Gt.device_bytes() > 0
    rt = Gt.solve(F, rtol=1e-8)
    torch.cuda.synchronize()
    with_state = torch.cuda.memory_allocated()
    Gh = _gpu(p, 3, allocator=None, **opts)
    rh = Gh.solve(F, rtol=1e-8)
    torch.cuda.synchronize()
    # the hipMalloc hierarchy and its state are invisible to torch: only u is
    # torch's (its caching allocator rounds blocks up to 512 bytes)
    assert torch.cuda.memory_allocated() - with_state == -(-rh.u.numel() * 8 // 512) * 512
    assert rt.converged and rh.converged and rt.iters == rh.iters
    assert torch.equal(rt.u, rh.u)
    Gh.close()
    Gt.close()
    del rt, rh
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


@pytest.mark.parametrize("smoother", [0, 2], ids=["jacobi", "chebyshev"])
@pytest.mark.parametrize("n_rhs", [1, 4])
def test_plan_bytes_cover_hierarchy_and_solve_state(smoother, n_rhs):
    from paper_2001_01655_amd import _lib as L
    print(f"plan bytes smoother={smoother} n_rhs={n_rhs}", flush=True)
    p = synth.small_case(3, (24, 16, 16), seed=62, n_rhs=n_rhs)
    F = torch.tensor(p.loads, device="cuda")
    U = torch.empty_like(F)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    G = _gpu(p, 3, smoother=smoother, nu_pre=2, nu_post=2, allocator="torch")
    G.solve(F, rtol=1e-8, out=U)
    torch.cuda.synchronize()
    used = torch.cuda.memory_allocated() - base
    plan = L.tm_plan_bytes(G.mesh, G.opts, n_rhs)
    print(f"  plan {plan} used {used} (hierarchy {G.device_bytes()})", flush=True)
    assert plan >= used
    G.close()


@pytest.mark.parametrize("kind,nel,ngeo", [("bridge", (32, 16, 16), 2), ("bridge", (32, 16, 16), 3),
                                           ("small", (64, 32), 2), ("small", (24, 16, 16), 2)])
def test_plan_bytes_cover_hybrid_hierarchies(kind, nel, ngeo):
    """Aggregation levels have data-dependent sizes: the plan's allowance for
    them (a dense coarsest level of up to 8 max_coarse dofs) covers what the
    hierarchy, its aggregation arenas and a two-load-case solve take."""
    from paper_2001_01655_amd import Hierarchy, _lib as L
    print(f"plan bytes hybrid {kind} {nel} ngeo={ngeo}", flush=True)
    p = synth.bridge_3d(nel=nel) if kind == "bridge" else synth.small_case(len(nel), nel, seed=62, n_rhs=2)
    F = torch.tensor(np.vstack([p.loads[0], p.loads[0]]), device="cuda")
    U = torch.empty_like(F)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    G = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_geometric=ngeo, max_coarse=300,
                  smoother=2, nu_pre=2, nu_post=2, cheb_warm_steps=4, allocator="torch")
    G.solve(F, rtol=1e-6, out=U)
    torch.cuda.synchronize()
    used = torch.cuda.memory_allocated() - base
    plan = L.tm_plan_bytes(G.mesh, G.opts, 2)
    print(f"  plan {plan} used {used}", flush=True)
    assert plan >= used
    G.close()
