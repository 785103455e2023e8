"""Warm-started Chebyshev intervals over a design stream (option
cheb_warm_steps): after every density update the solve still reaches the
oracle's dense solution of that design, with at most a couple more iterations
than the hierarchy that re-estimates every interval from the fixed start."""
import numpy as np
import pytest

import synth
from oracle import fem, mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dim,nel,levels", [(2, (40, 24), 3), (3, (12, 8, 8), 3), (3, (11, 7, 5), 3)])
def test_warm_intervals_over_a_design_stream(dim, nel, levels):
    from paper_2001_01655_amd import Hierarchy
    print(f"warm chebyshev {nel}", flush=True)
    p = synth.small_case(dim, nel, seed=17)
    kw = dict(p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=levels, smoother=2, nu_pre=2, nu_post=2)
    Hw = Hierarchy(p.nel, p.rho, p.fixed, cheb_warm_steps=4, **kw)
    Hc = Hierarchy(p.nel, p.rho, p.fixed, **kw)
    f = torch.tensor(p.loads[0], device="cuda")
    KE = fem.element_stiffness(dim, p.nu)
    seq = synth.design_sequence(p.rho, p.nel, seed=17)
    for t in range(6):
        rho = seq(t)
        if t > 0:
            Hw.update_density(torch.tensor(rho, device="cuda"))
            Hc.update_density(torch.tensor(rho, device="cuda"))
        rw = Hw.solve(f, rtol=1e-10)
        rc = Hc.solve(f, rtol=1e-10)
        assert rw.converged and rc.converged
        K = fem.apply_dirichlet(fem.assemble(p.nel, fem.simp(rho, p.p, p.E0, p.Emin), KE), p.fixed)
        u = mg.dense_solve(K, p.loads[0])
        err = np.linalg.norm(rw.u.cpu().numpy() - u) / np.linalg.norm(u)
        print(f"  design {t}: iterations warm {rw.iters[0]} cold {rc.iters[0]}, rel.err {err:.1e}", flush=True)
        assert err <= 1e-7
        assert rw.iters[0] <= rc.iters[0] + 2
    Hw.close()
    Hc.close()


@pytest.mark.parametrize("variant", ["hybrid", "demotion"])
def test_warm_intervals_with_aggregation_levels(variant):
    """Warm intervals when aggregation levels exist (their estimates always
    start cold) and when the automated hybrid turns the last geometric level
    into aggregation levels mid-stream (that level's kept vector is no longer
    used): every design's u still equals the oracle's dense solve."""
    from paper_2001_01655_amd import Hierarchy
    print(f"warm chebyshev {variant}", flush=True)
    p = synth.small_case(3, (16, 8, 8), seed=19)
    kw = dict(p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, smoother=2, nu_pre=2, nu_post=2, cheb_warm_steps=4)
    if variant == "hybrid":
        kw.update(n_geometric=2, max_coarse=300)
    else:
        kw.update(n_levels=4, adapt_iters=1)      # every solve demotes one geometric level (down to 2)
    H = Hierarchy(p.nel, p.rho, p.fixed, **kw)
    f = torch.tensor(p.loads[0], device="cuda")
    KE = fem.element_stiffness(3, p.nu)
    seq = synth.design_sequence(p.rho, p.nel, seed=19)
    levels = []
    for t in range(4):
        rho = seq(t)
        if t > 0:
            H.update_density(torch.tensor(rho, device="cuda"))
        r = H.solve(f, rtol=1e-10)
        assert r.converged
        levels.append(H.num_levels())
        K = fem.apply_dirichlet(fem.assemble(p.nel, fem.simp(rho, p.p, p.E0, p.Emin), KE), p.fixed)
        u = mg.dense_solve(K, p.loads[0])
        err = np.linalg.norm(r.u.cpu().numpy() - u) / np.linalg.norm(u)
        print(f"  design {t}: {H.num_levels()} levels, iterations {r.iters[0]}, rel.err {err:.1e}", flush=True)
        assert err <= 1e-7
    H.close()
