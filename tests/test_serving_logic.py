"""Scheduling logic of the continuous-batching loop, on the CPU with a fake
engine (no device): admission by memory budget and slots, arrival order,
every design of every request solved in order, results independent of the
mix."""
import numpy as np
import pytest

from paper_2001_01655_amd.serving import Request, Server


class FakeState:
    def __init__(self, key, need):
        self.key = key
        self.left = need          # iterations still needed
        self.inflight = 0
        self.advanced = 0


class FakeResult:
    def __init__(self, iters, comp, u):
        self.iters = iters
        self.compliance = comp
        self.status = 0
        self.u = u


class FakeEngine:
    """Deterministic stand-in: a solve needs a number of iterations fixed by
    (request, design); 'compliance' depends only on the request, the design
    and the warm start it was given."""

    def __init__(self):
        self.live = 0
        self.max_live = 0
        self.log = []

    def plan_bytes(self, req):
        return 100 * int(np.prod(req.nel))

    def new_stream(self):
        return object()

    def setup(self, req, rho, stream):
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        return {"req": req, "design": 0, "rho": float(np.sum(rho))}

    def update(self, h, rho, stream):
        h["design"] += 1
        h["rho"] = float(np.sum(rho))

    def begin(self, h, req, rtol, u0, stream):
        need = 3 + (req.rid * 7 + h["design"] * 3) % 5
        st = FakeState((req.rid, h["design"]), need)
        st.u0 = 0.0 if u0 is None else u0
        st.h = h
        self.log.append(("begin", req.rid, h["design"]))
        return st

    def poll(self, st):
        if st.inflight:
            st.inflight = 0            # the enqueued chunk completes between polls
            return 1 if st.left <= 0 else 0
        return 1 if st.left <= 0 else 0

    def batch_advance(self, states, k):
        for st in states:
            st.left -= k
            st.inflight = 1
            st.advanced += k

    def end(self, st):
        rid, d = st.key
        c = st.h["rho"] + 0.5 * st.u0 + rid
        return FakeResult([st.advanced], [c], c)

    def release(self, h):
        self.live -= 1


def _reqs(n, designs=3, spacing=0.0):
    out = []
    for rid in range(n):
        nel = (8 + 4 * (rid % 3), 4 + 2 * (rid % 2))
        rho = np.full(int(np.prod(nel)), 0.5 + 0.01 * rid)
        out.append(Request(rid, spacing * rid, nel, np.array([0]), np.zeros((1 + rid % 2, 10)),
                           lambda t, rho=rho: rho * (1 + 0.1 * t), designs))
    return out


def test_all_designs_solved_in_order_and_budget_respected():
    eng = FakeEngine()
    reqs = _reqs(9)
    budget = 100 * 16 * 6 * 2          # room for about two of the larger requests
    srv = Server(eng, hbm_budget=budget, max_slots=3, chunk=2)
    out = srv.run(reqs)
    assert [o.rid for o in out["outcomes"]] == list(range(9))
    assert srv.peak_in_use <= budget
    assert eng.max_live <= 3
    for o in out["outcomes"]:
        assert len(o.iters) == 3 and len(o.compliance) == 3
    for rid in range(9):
        seq = [d for (ev, r, d) in eng.log if r == rid]
        assert seq == [0, 1, 2]
    assert out["solves"] == sum(r.n_rhs * 3 for r in reqs)
    assert out["p99_ms"] >= out["p50_ms"] >= 0.0


def test_results_same_alone_and_in_mix():
    reqs = _reqs(6)
    mix = Server(FakeEngine(), hbm_budget=10 ** 9, max_slots=4, chunk=3).run(reqs)
    for r in reqs:
        alone = Server(FakeEngine(), hbm_budget=10 ** 9, max_slots=1, chunk=3).run([r])
        a = alone["outcomes"][0]
        m = mix["outcomes"][r.rid]
        assert a.compliance == m.compliance and a.iters == m.iters


def test_overlap_and_arrival_order():
    eng = FakeEngine()
    t = [0.0]

    def clock():
        t[0] += 1e-4
        return t[0]

    reqs = _reqs(5, designs=4, spacing=2e-3)
    out = Server(eng, hbm_budget=10 ** 9, max_slots=8, chunk=1).run(reqs, clock=clock)
    assert eng.max_live >= 2                     # requests overlap on the device
    adm = [o.admitted for o in out["outcomes"]]
    assert all(o.admitted >= o.arrival for o in out["outcomes"])
    assert adm == sorted(adm)


def test_oversized_request_rejected():
    eng = FakeEngine()
    with pytest.raises(ValueError):
        Server(eng, hbm_budget=10, max_slots=2).run(_reqs(1))


class LaggingEngine(FakeEngine):
    """A chunk stays in flight for a few polls (poll returns -1 meanwhile);
    records how many chunks were still running at every grouped call."""

    def __init__(self, lag):
        super().__init__()
        self.lag = lag
        self.running = set()
        self.calls = []

    def poll(self, st):
        if st.inflight:
            st.inflight -= 1
            if st.inflight:
                return -1
            self.running.discard(id(st))
        return 1 if st.left <= 0 else 0

    def batch_advance(self, states, k):
        self.calls.append((len(states), len(self.running)))
        for st in states:
            st.left -= k
            st.inflight = 1 + self.lag
            st.advanced += k
            self.running.add(id(st))


@pytest.mark.parametrize("gather", [0.0, 1.0, float("inf")])
def test_gathering_idle_solves(gather):
    """With gather g, idle solves advance while others run only when they are
    at least g times as many; the default (infinite) advances only when nothing
    runs.  Results never depend on it."""
    reqs = _reqs(6, designs=3)
    eng = LaggingEngine(lag=3)
    out = Server(eng, hbm_budget=10 ** 9, max_slots=6, chunk=2, gather=gather).run(reqs)
    ref = Server(FakeEngine(), hbm_budget=10 ** 9, max_slots=6, chunk=2).run(reqs)
    for a, b in zip(out["outcomes"], ref["outcomes"]):
        assert a.compliance == b.compliance and a.iters == b.iters
    for n_idle, n_running in eng.calls:
        assert n_running == 0 or n_idle >= gather * n_running
    if gather == float("inf"):
        assert all(r == 0 for _, r in eng.calls)
