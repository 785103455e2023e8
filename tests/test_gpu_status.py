"""The solve's failure statuses on the GPU: each ends the solve with a status
(no fault, no hang), and the hierarchy and device stay usable afterwards.

  * TM_NOT_CONVERGED: the iteration limit is reached; u is the last iterate.
  * TM_ERR_BREAKDOWN: standard PCG meets z^T r <= 0, which happens when the
    V-cycle is not positive definite.  Over-relaxed block Jacobi (omega 1.99,
    3 sweeps) makes it so; the oracle's V-cycle confirms that z^T r of the
    first residual is clearly negative for the same inputs.
  * TM_ERR_ARG from non-finite data: a load with a NaN or an infinity is
    refused by the solve's first step (||f||^2 or ||r_0||^2 not finite).
  * A singular operator (no supports: the rigid-body motions are free) is
    reported as not positive definite by the coarsest factorisation or stops the
    solve with a failure status; it never reports success.
"""
import numpy as np
import pytest

import synth
from oracle import fem, mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _gpu(p, L, **kw):
    from paper_2001_01655_amd import Hierarchy
    return Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=L, **kw)


def _good_solve_after(G, p):
    r = G.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-8)
    return r


@pytest.mark.parametrize("vfp,outer", [(32, 0), (64, 1)])
def test_not_converged(vfp, outer):
    from paper_2001_01655_amd import _lib as L
    _say(f"not converged vfp={vfp}")
    p = synth.small_case(3, (12, 8, 8), seed=41)
    G = _gpu(p, 3, vcycle_fp=vfp, outer=outer, max_iters=3)
    r = G.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-10)
    u = r.u.cpu().numpy()
    assert r.status == L.TM_NOT_CONVERGED and not r.converged
    assert r.iters[0] == 3
    assert np.isfinite(r.relres[0]) and r.relres[0] > 1e-10
    assert np.all(np.isfinite(u)) and np.all(u[p.fixed] == 0.0)
    # the reported residual is the true one of the last iterate
    KE = fem.element_stiffness(3, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    f = p.loads[0].copy()
    f[p.fixed] = 0.0
    rel = np.linalg.norm(f - fem.apply_matfree(p.nel, E, KE, p.fixed, u)) / np.linalg.norm(f)
    assert abs(rel - r.relres[0]) <= 1e-6 * rel
    G.close()


@pytest.mark.parametrize("dim,nel", [(3, (12, 8, 8)), (2, (28, 12))])
def test_breakdown_indefinite_vcycle(dim, nel):
    from paper_2001_01655_amd import TmError
    from paper_2001_01655_amd import _lib as L
    _say(f"breakdown omega 1.99 {nel}")
    p = synth.small_case(dim, nel, seed=41)
    f = p.loads[0].copy()
    f[p.fixed] = 0.0
    # the oracle's V-cycle with the same smoother: z^T r < 0 for r = f
    KE = fem.element_stiffness(dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    H = mg.build_geometric(p.nel, E, KE, p.fixed, 3, omega=1.99, nu_pre=3, nu_post=3)
    z = mg.vcycle(H, f)
    assert f @ z < -0.05 * np.linalg.norm(f) * np.linalg.norm(z)
    G = _gpu(p, 3, omega=1.99, nu_pre=3, nu_post=3, vcycle_fp=64, outer=L.TM_OUTER_PCG)
    with pytest.raises(TmError) as e:
        G.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-8)
    assert e.value.status == L.TM_ERR_BREAKDOWN
    G.close()
    # a sound hierarchy on the same device solves normally afterwards
    G = _gpu(p, 3)
    assert _good_solve_after(G, p).converged
    G.close()


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
def test_nonfinite_load(bad):
    from paper_2001_01655_amd import TmError
    from paper_2001_01655_amd import _lib as L
    _say(f"non-finite load {bad}")
    p = synth.small_case(3, (12, 8, 8), seed=42)
    G = _gpu(p, 3)
    f = p.loads[0].copy()
    free = np.setdiff1d(np.arange(p.n_dof), p.fixed)
    f[free[len(free) // 2]] = bad
    with pytest.raises(TmError) as e:
        G.solve(torch.tensor(f, device="cuda"), rtol=1e-8)
    assert e.value.status == L.TM_ERR_ARG and "not finite" in str(e.value)
    # the same hierarchy solves a finite load afterwards
    assert _good_solve_after(G, p).converged
    G.close()


def test_singular_operator_is_not_reported_as_solved():
    from paper_2001_01655_amd import Hierarchy, TmError
    from paper_2001_01655_amd import _lib as L
    _say("no supports")
    p = synth.small_case(2, (16, 8), seed=43)
    f = torch.tensor(p.loads[0], device="cuda")
    status = None
    try:
        G = Hierarchy(p.nel, p.rho, np.zeros(0, dtype=np.int64), p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu,
                      n_levels=3, max_iters=200)
    except TmError as e:
        status = e.status
    else:
        try:
            status = G.solve(f, rtol=1e-8).status
        except TmError as e:
            status = e.status
        G.close()
    _say(f"  status {status}")
    assert status in (L.TM_ERR_NOT_SPD, L.TM_ERR_BREAKDOWN, L.TM_NOT_CONVERGED)
    G = _gpu(p, 3)
    assert _good_solve_after(G, p).converged
    G.close()
