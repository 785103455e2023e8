"""Served stream on the GPU: requests of different meshes and load-case
counts run concurrently (one stream each, batched iteration) and every
result equals the result of the same request run alone."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mix(n_designs=3):
    from paper_2001_01655_amd.serving import Request
    sizes = [(2, (32, 16)), (3, (8, 8, 8)), (2, (64, 32)), (3, (16, 8, 8)), (2, (32, 16)), (3, (8, 8, 8))]
    reqs = []
    for rid, (dim, nel) in enumerate(sizes):
        n_rhs = 1 + rid % 3
        rho0 = synth.minmax_density(synth.smoothed_field(tuple(reversed(nel)), 50 + rid, sigma=2.0)).ravel()
        dens = synth.design_sequence(rho0, nel, 60 + rid)

        reqs.append(Request(rid, 0.001 * rid, nel, synth.clamp_x0(nel, dim), synth.served_loads(nel, dim, n_rhs),
                            dens, n_designs, options=dict(max_coarse=100)))
    return reqs


def test_mix_equals_alone():
    from paper_2001_01655_amd.serving import GpuEngine, Server
    eng = GpuEngine()
    reqs = _mix()
    mix = Server(eng, hbm_budget=8 << 30, max_slots=4, chunk=3, rtol=1e-6, keep_solutions=True).run(reqs)
    print("mix:", {k: v for k, v in mix.items() if k != "outcomes"}, flush=True)
    assert len(mix["outcomes"]) == len(reqs)
    for r in reqs:
        alone = Server(eng, hbm_budget=8 << 30, max_slots=1, chunk=5, rtol=1e-6, keep_solutions=True).run([r])
        a, m = alone["outcomes"][0], mix["outcomes"][r.rid]
        assert all(s == 0 for s in m.status)
        for ca, cm in zip(a.compliance, m.compliance):
            np.testing.assert_allclose(cm, ca, rtol=1e-12, atol=0)
        ua, um = a.u_last.cpu().numpy(), m.u_last.cpu().numpy()
        assert np.max(np.abs(ua - um)) <= 1e-12 * np.max(np.abs(ua))


def test_served_stream_runs():
    from paper_2001_01655_amd.serving import GpuEngine, Server, served_requests
    reqs = served_requests(4, rate_per_s=50.0, n_designs=2)
    out = Server(GpuEngine(), hbm_budget=16 << 30, max_slots=4, chunk=4, rtol=1e-6).run(reqs)
    assert len(out["outcomes"]) == 4
    for o in out["outcomes"]:
        assert all(s == 0 for s in o.status)
        assert all(len(c) == reqs[o.rid].n_rhs for c in o.compliance)
    print("served:", {k: v for k, v in out.items() if k != "outcomes"}, flush=True)
