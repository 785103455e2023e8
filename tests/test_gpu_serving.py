"""Served stream on the GPU: requests of different meshes and load-case
counts run concurrently (one stream each, batched iteration) and every
result equals the result of the same request run alone."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _mix(n_designs=3, hybrid=False):
    """Requests of several sizes, repeated sizes among them (their load cases
    share launches in the mix), 1-3 load cases; optionally one hybrid request
    (smoothed aggregation below two geometric levels)."""
    from paper_2001_01655_amd.serving import Request
    sizes = [(2, (32, 16)), (3, (8, 8, 8)), (2, (64, 32)), (3, (16, 8, 8)), (2, (32, 16)), (3, (8, 8, 8))]
    if hybrid:
        sizes.append((3, (16, 8, 8)))
    reqs = []
    for rid, (dim, nel) in enumerate(sizes):
        n_rhs = 1 + rid % 3
        rho0 = synth.minmax_density(synth.smoothed_field(tuple(reversed(nel)), 50 + rid, sigma=2.0)).ravel()
        dens = synth.design_sequence(rho0, nel, 60 + rid)
        opts = dict(max_coarse=100)
        if hybrid and rid == len(sizes) - 1:
            opts.update(n_geometric=2)
        reqs.append(Request(rid, 0.001 * rid, nel, synth.clamp_x0(nel, dim), synth.served_loads(nel, dim, n_rhs),
                            dens, n_designs, options=opts))
    return reqs


SERVED = dict(smoother=2, nu_pre=2, nu_post=2, cheb_warm_steps=4)


@pytest.mark.parametrize("engine_opts,hybrid", [({}, False), (SERVED, True)], ids=["jacobi", "served_with_hybrid"])
def test_mix_equals_alone(engine_opts, hybrid):
    """Every request's compliances and last displacements are the same in the
    mix (grouped launches with other requests) as alone."""
    from paper_2001_01655_amd.serving import GpuEngine, Server
    print(f"mix equals alone {engine_opts} hybrid={hybrid}", flush=True)
    eng = GpuEngine(**engine_opts)
    reqs = _mix(hybrid=hybrid)
    mix = Server(eng, hbm_budget=8 << 30, max_slots=4, chunk=3, rtol=1e-6, keep_solutions=True,
                 workers=2).run(reqs)
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
        assert a.iters == m.iters


def test_served_stream_runs():
    from paper_2001_01655_amd.serving import GpuEngine, Request, Server
    arrivals = synth.poisson_arrivals(4, 50.0, 5)
    reqs = []
    for rid in range(4):
        p = synth.served_request(rid, 5)
        reqs.append(Request(rid, float(arrivals[rid]), p.nel, p.fixed, p.loads,
                            synth.design_sequence(p.rho, p.nel, 5 + rid), 2,
                            material=dict(p=p.p, E0=p.E0, Emin=p.Emin, nu=p.nu)))
    out = Server(GpuEngine(), hbm_budget=16 << 30, max_slots=4, chunk=4, rtol=1e-6).run(reqs)
    assert len(out["outcomes"]) == 4
    for o in out["outcomes"]:
        assert all(s == 0 for s in o.status)
        assert all(len(c) == reqs[o.rid].n_rhs for c in o.compliance)
    print("served:", {k: v for k, v in out.items() if k != "outcomes"}, flush=True)


def test_batch_iterate_groups_equal_alone():
    """tm_batch_iterate over states of hierarchies with the same level
    structure (grouped launches) and one of another shape: every solution is
    bitwise the solution of the same hierarchy solved alone."""
    from paper_2001_01655_amd import Hierarchy
    from paper_2001_01655_amd.solver import tm_batch_iterate
    print("batch iterate", flush=True)
    cases = [(3, (12, 8, 8), 71, 2), (3, (12, 8, 8), 72, 1), (3, (12, 8, 8), 73, 3), (2, (40, 20), 74, 2)]
    Hs, Fs, alone = [], [], []
    for dim, nel, seed, n_rhs in cases:
        p = synth.small_case(dim, nel, seed=seed, n_rhs=n_rhs)
        H = Hierarchy(p.nel, p.rho, p.fixed, n_levels=3, smoother=2, nu_pre=2, nu_post=2)
        F = torch.tensor(p.loads, device="cuda")
        alone.append(H.solve(F, rtol=1e-8))
        Hs.append(H)
        Fs.append(F)
    stream = torch.cuda.Stream()
    states = [H.begin(F, 1e-8) for H, F in zip(Hs, Fs)]
    for _ in range(200):
        live = [s for s in states if s.poll() != 1]
        if not live:
            break
        tm_batch_iterate(live, 3, stream)
        torch.cuda.synchronize()
    for s, a in zip(states, alone):
        r = s.end()
        assert r.converged and r.iters == a.iters
        assert torch.equal(r.u, a.u)
    for H in Hs:
        H.close()


def _outputs_match_definition(H, F, r):
    """compliance f^T u and relres ||f - K~u|| / ||f|| of every load case, K~u
    from tm_apply (FP64, a different summation order than the solve's own)."""
    for k in range(F.shape[0]):
        f, u = F[k].double(), r.u[k].double()
        c = float(torch.dot(f, u))
        rel = float(torch.linalg.norm(f - H.apply(0, u)) / torch.linalg.norm(f))
        assert abs(r.compliance[k] - c) <= 1e-12 * abs(c)
        assert abs(r.relres[k] - rel) <= 1e-3 * rel + 1e-13


def test_end_outputs_left_by_the_last_batch():
    """The outputs that a batch leaves for the load cases that stopped in it
    (and that begin leaves for a start already within the tolerance) are the
    true residual and compliance of the returned displacements; a state ended
    before it stopped computes them at end with the same kernels."""
    from paper_2001_01655_amd import Hierarchy
    from paper_2001_01655_amd.solver import tm_batch_iterate
    print("end outputs", flush=True)
    p = synth.small_case(3, (12, 8, 8), seed=75, n_rhs=2)
    H = Hierarchy(p.nel, p.rho, p.fixed, n_levels=3)
    F = torch.tensor(p.loads, device="cuda")
    stream = torch.cuda.Stream()
    st = H.begin(F, 1e-8)
    for _ in range(200):
        if st.poll() == 1:
            break
        tm_batch_iterate([st], 2, stream)
        torch.cuda.synchronize()
    r = st.end()
    assert r.converged
    _outputs_match_definition(H, F, r)
    a = H.solve(F, rtol=1e-8)
    assert r.iters == a.iters and r.compliance == a.compliance and r.relres == a.relres
    # start within the tolerance: no iteration, outputs from begin
    st = H.begin(F, 1e-6, u0=r.u)
    torch.cuda.synchronize()
    assert st.poll() == 1
    w = st.end()
    assert w.converged and w.iters == [0, 0]
    _outputs_match_definition(H, F, w)
    # ended after one iteration, before stopping: outputs computed by end
    st = H.begin(F, 1e-12)
    tm_batch_iterate([st], 1, stream)
    torch.cuda.synchronize()
    assert st.poll() == 0
    e = st.end()
    assert e.iters == [1, 1]
    _outputs_match_definition(H, F, e)
    H.close()
