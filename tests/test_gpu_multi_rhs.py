"""Several load cases in one solve (the adjoint solves of Sec. 2 with x0 = 0):
all right-hand sides share each launch, and on the stored-stencil levels one
thread serves up to four of them, reading the level's operator and block
inverse once.  Every load case's solution and iteration count are bitwise
those of its own single-load-case solve."""
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

OPTS = {
    "jacobi": dict(),
    "chebyshev": dict(smoother=2, nu_pre=2, nu_post=2),
    "fp64_pcg": dict(vcycle_fp=64, outer=1),
}


def _check(p, n_levels, **opts):
    from paper_2001_01655_amd import Hierarchy
    H = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=n_levels, **opts)
    F = torch.tensor(p.loads, device="cuda")
    r = H.solve(F, rtol=1e-8)
    assert r.converged
    for k in range(F.shape[0]):
        a = H.solve(F[k], rtol=1e-8)
        assert a.iters[0] == r.iters[k], (k, a.iters, r.iters)
        assert torch.equal(a.u.reshape(-1), r.u[k].reshape(-1)), k
        assert a.compliance[0] == r.compliance[k]
    H.close()


@pytest.mark.parametrize("n_rhs", [2, 3, 5, 6, 9])
@pytest.mark.parametrize("opt", list(OPTS))
@pytest.mark.parametrize("dim,nel,L", [(3, (16, 8, 8), 3), (2, (48, 24), 4), (3, (11, 7, 5), 3)])
def test_load_cases_equal_single_solves(dim, nel, L, opt, n_rhs):
    """Small grids with the large-level stencil kernel on every level (option
    stencil_kernel = 1), so that the shared-operator form runs on every coarse
    level; 9 load cases span two launches of up to 8 lanes."""
    print(f"multi-rhs {dim}D {nel} {opt} n_rhs={n_rhs}", flush=True)
    p = synth.small_case(dim, nel, seed=40 + n_rhs, n_rhs=n_rhs)
    _check(p, L, stencil_kernel=1, **OPTS[opt])


def test_load_cases_at_large_level_size():
    """3D 128x64x64: level 1 (70,785 nodes) selects the large-level kernel by
    size; six load cases (two groups of three per thread)."""
    print("multi-rhs 3D (128, 64, 64) chebyshev n_rhs=6", flush=True)
    p = synth.small_case(3, (128, 64, 64), seed=47, n_rhs=6)
    _check(p, 5, **OPTS["chebyshev"])
