"""The configurations at full size on the GPU, checked by properties the
oracle evaluates at any size: true residual from the oracle's own element sum,
compliance identity, supports, and agreement of the FP32-V-cycle and
FP64-everywhere solutions."""
import numpy as np
import pytest

import synth
from oracle import fem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (problem, options); the Chebyshev 2/2 cantilever is the benchmark's configuration
CHEB22 = dict(smoother=2, nu_pre=2, nu_post=2)
CONFIGS = {
    "cantilever2d": ("cantilever2d", dict(n_levels=7, max_iters=20000)),
    "cantilever3d": ("cantilever3d", dict(n_levels=6)),
    "cantilever3d_cheb": ("cantilever3d", dict(n_levels=6, **CHEB22)),
    "bridge3d": ("bridge3d", dict(n_geometric=3, max_coarse=1000)),
    # Sec. 4.3: 5 geometric levels with ceil(n/2) coarsening, 2312 coarsest dofs
    "grid2d": ("grid2d", dict(n_levels=5, max_iters=20000)),
}


def _check(p, res, k=0):
    u = res.u.cpu().numpy().reshape(-1, p.n_dof)[k]
    f = p.loads[k].copy()
    f[p.fixed] = 0.0
    KE = fem.element_stiffness(p.dim, p.nu)
    E = fem.simp(p.rho, p.p, p.E0, p.Emin)
    r = f - fem.apply_matfree(p.nel, E, KE, p.fixed, u)
    rel = np.linalg.norm(r) / np.linalg.norm(f)
    print(f"  {p.name}: iters={res.iters[k]} oracle true relres={rel:.3e} (gpu {res.relres[k]:.3e})", flush=True)
    # the GPU reports the true residual of its FP64 operator; the two element
    # sums differ only by rounding, which is far below the tolerance
    assert rel <= 2e-8 and res.relres[k] <= 2e-8
    assert abs(rel - res.relres[k]) <= 0.05 * rel
    assert abs(res.compliance[k] - f @ u) <= 1e-12 * abs(f @ u)
    assert np.all(u[p.fixed] == 0.0)
    return u


@pytest.mark.parametrize("name", list(CONFIGS))
def test_full_size_solve(name):
    from paper_2001_01655_amd import Hierarchy
    print(f"full size {name}", flush=True)
    prob, opts = CONFIGS[name]
    p = synth.get(prob)
    H = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, **opts)
    res = H.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-8)
    assert res.status == 0
    _check(p, res)
    if name == "grid2d":
        sizes = [H.level_info(l)["n_rows"] for l in range(H.num_levels())]
        assert sizes == [2 * 521 * 521, 2 * 261 * 261, 2 * 131 * 131, 2 * 66 * 66, 2312]
    if name == "bridge3d":
        info = [H.level_info(l) for l in range(H.num_levels())]
        lg = next(l for l, i in enumerate(info) if i["kind"] == 2) - 1
        agg = H.export_aggregates(lg)
        n_agg = info[lg + 1]["n_rows"] // info[lg + 1]["block"]
        assert agg.min() == 0 and agg.max() == n_agg - 1
        assert np.all(np.bincount(agg, minlength=n_agg) > 0)
    H.close()


@pytest.mark.parametrize("opts", [{}, CHEB22], ids=["jacobi", "chebyshev"])
def test_mixed_equals_fp64_at_full_size(opts):
    from paper_2001_01655_amd import Hierarchy
    p = synth.get("cantilever3d")
    f = torch.tensor(p.loads[0], device="cuda")
    us = []
    for vfp, outer in [(32, 0), (64, 1)]:
        H = Hierarchy(p.nel, p.rho, p.fixed, n_levels=6, vcycle_fp=vfp, outer=outer, **opts)
        r = H.solve(f, rtol=1e-8)
        assert r.status == 0
        us.append(r.u.clone())
        H.close()
    d = float((us[0] - us[1]).norm() / us[1].norm())
    print(f"  mixed vs fp64: {d:.2e}", flush=True)
    assert d <= 1e-7


# ---------------------------------------------------------------- against the oracle's solutions
# golden case -> (problem, GPU options); the oracle's u at rtol 1e-12 comes
# from tests/golden/make_golden.py (oracle only)
import json  # noqa: E402
import os  # noqa: E402

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GOLDEN = {
    "mbb_random": (lambda: synth.mbb_2d(False), dict(n_levels=3, omega=0.6, nu_pre=2, nu_post=2)),
    "grid2d": (lambda: synth.get("grid2d"), dict(n_levels=5, max_iters=20000)),
    "cantilever2d": (lambda: synth.get("cantilever2d"), dict(n_levels=7, max_iters=20000)),
    "cantilever3d": (lambda: synth.get("cantilever3d"), dict(n_levels=6)),
    "cantilever3d_cheb": (lambda: synth.get("cantilever3d"), dict(n_levels=6, **CHEB22)),
    # the bridge recipe at an eighth of its volume (the oracle's aggregation
    # levels at full size do not fit in a workstation's memory)
    "bridge3d_128x64x64": (lambda: synth.bridge_3d(nel=(128, 64, 64)), dict(n_geometric=3, max_coarse=1000)),
}


def golden_errors(g, u, c):
    """Relative errors of a solution against an oracle reference: u over the
    sampled dofs, ||u||_2, and the compliance."""
    idx = np.asarray(g["sample_dofs"], dtype=np.int64)
    ref = np.asarray(g["sample_u"])
    e_u = float(np.linalg.norm(u[idx] - ref) / np.linalg.norm(ref))
    e_n = abs(float(np.linalg.norm(u)) - g["norm_u"]) / g["norm_u"]
    e_c = abs(c - g["compliance"]) / abs(g["compliance"])
    return e_u, e_n, e_c


@pytest.mark.parametrize("name", list(GOLDEN))
def test_full_size_vs_oracle(name):
    """FP32-V-cycle / FP64-FCG solve at rtol 1e-8 against the oracle's u at
    rtol 1e-12: relative error <= 1e-7 over 4096 seeded dofs and in ||u||,
    and <= 1e-9 in the compliance.  Where the oracle's true residual stays
    above 1e-11 (the FP64 floor eps ||K|| ||u|| / ||f|| of a 1e9 stiffness
    contrast: restarts no longer lower it), its compliance is itself only
    known to about that residual, and the compliance bound is ten times the
    reference's true relative residual."""
    from paper_2001_01655_amd import Hierarchy
    path = os.path.join(GOLDEN_DIR, f"solve_{name.replace('_cheb', '')}.json")
    with open(path) as fh:
        g = json.load(fh)
    make, opts = GOLDEN[name]
    p = make()
    fp = g["inputs"]
    assert fp["n_dof"] == p.n_dof and fp["n_fixed"] == len(p.fixed)
    assert abs(fp["rho_sum"] - float(np.sum(p.rho))) <= 1e-12 * abs(fp["rho_sum"]), "density generator changed"
    assert fp["load_sum"] == float(np.sum(p.loads[0])), "load generator changed"
    print(f"vs oracle {name} ({p.n_dof} dofs)", flush=True)
    H = Hierarchy(p.nel, p.rho, p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, **opts)
    res = H.solve(torch.tensor(p.loads[0], device="cuda"), rtol=1e-8)
    H.close()
    assert res.status == 0
    u = res.u.cpu().numpy().reshape(-1)
    e_u, e_n, e_c = golden_errors(g, u, res.compliance[0])
    print(f"  iters={res.iters[0]} err_u(sampled)={e_u:.2e} err_norm={e_n:.2e} err_c={e_c:.2e}", flush=True)
    tol_c = max(1e-9, 10.0 * g["oracle"]["true_relres"])
    assert e_u <= 1e-7 and e_n <= 1e-7 and e_c <= tol_c
