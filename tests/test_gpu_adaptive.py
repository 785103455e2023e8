"""The automated hybrid (second hybrid of Sec. 4.4) on the GPU against the
oracle's stream: the level structure used for each design, and each design's
solution, through tm_setup / tm_solve / tm_update_density."""
import numpy as np
import pytest

import synth
from oracle import adaptive

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _stream(dim, nel, n, seed):
    p = synth.small_case(dim, nel, seed=seed)
    rhos = [p.rho]
    for t in range(1, n):
        rhos.append(synth.density_update(rhos[-1], p.nel, seed=seed, step=t))
    return p, rhos


@pytest.mark.parametrize("dim,nel,G0,max_coarse,threshold", [
    (3, (8, 4, 4), 3, 100, 1),            # drops to two geometric levels + aggregation
    (3, (16, 8, 8), 4, 300, 1),
    (2, (64, 32), 5, 200, 1),
    (3, (16, 8, 8), 4, 300, 10 ** 6),     # never reached: stays geometric
])
def test_adaptive_stream_matches_oracle(dim, nel, G0, max_coarse, threshold):
    from paper_2001_01655_amd import Hierarchy
    print(f"adaptive stream {nel} G0={G0} threshold={threshold}", flush=True)
    p, rhos = _stream(dim, nel, 4, seed=52)
    ref = adaptive.adaptive_stream(p.nel, rhos, p.fixed, p.loads[0], n_start=G0, threshold=threshold,
                                   max_coarse=max_coarse)
    H = Hierarchy(p.nel, rhos[0], p.fixed, p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu, n_levels=G0,
                  max_coarse=max_coarse, adapt_iters=threshold, vcycle_fp=64, outer=1)
    f = torch.tensor(p.loads[0], device="cuda")
    for t, (rho, s) in enumerate(zip(rhos, ref)):
        if t:
            H.update_density(torch.tensor(rho, device="cuda"))
        r = H.solve(f, rtol=1e-8)
        kinds = [H.level_info(l)["kind"] for l in range(H.num_levels())]
        n_geo = sum(k != 2 for k in kinds)
        u = r.u.cpu().numpy()
        e = np.linalg.norm(u - s.u) / np.linalg.norm(s.u)
        print(f"  design {t}: geometric {n_geo} (oracle {s.n_geometric}), levels {len(kinds)} "
              f"(oracle {s.levels}), iters {r.iters[0]} (oracle {s.iters}), err_u {e:.2e}", flush=True)
        assert r.converged
        assert n_geo == s.n_geometric and len(kinds) == s.levels
        assert e <= 1e-7
    H.close()
