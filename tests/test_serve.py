"""Serving loop scheduling, against a fake backend on a virtual clock.

The fake backend implements the same case API as the GPU backend
(footprint / create / advance / finish); advancing a group of cases costs
virtual time, so admission, arrival order, the memory budget and continuous
batching can be checked exactly on the CPU.
"""
import dataclasses

import pytest

from paper_1207_1571_amd.serve import Request, Server, summarize


@dataclasses.dataclass
class _Mesh:
    n_cells: int


@dataclasses.dataclass
class _Spec:
    mesh: _Mesh


class FakeBackend:
    """Each group advance costs `step_cost` virtual seconds per step plus a
    per-launch overhead; records residency to check the budget."""

    def __init__(self, clock, bytes_per_cell=600, step_cost=1e-3, overhead=1e-4, fail_rid=None):
        self.clock = clock
        self.bpc = bytes_per_cell
        self.step_cost = step_cost
        self.overhead = overhead
        self.fail_rid = fail_rid
        self.resident = {}
        self.max_resident_bytes = 0
        self.max_resident_cases = 0
        self.groups = []
        self.created_at = {}

    def footprint(self, spec):
        return spec.mesh.n_cells * self.bpc

    def create(self, spec):
        case = object()
        self.resident[id(case)] = self.footprint(spec)
        self.created_at[id(case)] = self.clock.t
        self.max_resident_bytes = max(self.max_resident_bytes, sum(self.resident.values()))
        self.max_resident_cases = max(self.max_resident_cases, len(self.resident))
        case_spec[id(case)] = spec
        return case

    def advance(self, cases, n_steps):
        self.groups.append((self.clock.t, len(cases), n_steps))
        self.clock.t += self.overhead + n_steps * self.step_cost
        out = []
        for c in cases:
            rid = getattr(case_spec[id(c)], "rid", None)
            st = -3 if rid is not None and rid == self.fail_rid else 0
            out.append({"p": [{"iters": 5}] * n_steps, "status": st})
        return out

    def finish(self, case):
        del self.resident[id(case)]
        return None


case_spec = {}


class VClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


def _spec(n_cells, rid=None):
    s = _Spec(_Mesh(n_cells))
    if rid is not None:
        s.rid = rid
    return s


def _server(backend, clock, budget, **kw):
    return Server(backend, budget, clock=clock, sleep=clock.sleep, **kw)


def test_all_requests_complete_and_latency_accounts_steps():
    clk = VClock()
    be = FakeBackend(clk)
    reqs = [Request(i, 0.01 * i, _spec(1000 + 10 * i), 20) for i in range(12)]
    res = _server(be, clk, 10**9, slots=4, group=2, chunk=5).run(reqs)
    assert sorted(r.rid for r in res) == list(range(12))
    for r in res:
        assert r.admitted_s >= r.arrival_s
        assert r.done_s > r.admitted_s
        # every case needs at least n_steps steps of its own group
        assert r.latency_s >= 20 * be.step_cost
        assert r.p_iters == 5 * 20
        assert r.status == 0
    s = summarize(res)
    assert s["n"] == 12 and s["failed"] == 0
    assert s["p50_s"] <= s["p99_s"] <= s["max_s"]


def test_arrivals_are_honoured():
    clk = VClock()
    be = FakeBackend(clk)
    reqs = [Request(0, 0.0, _spec(100), 3), Request(1, 5.0, _spec(100), 3)]
    res = {r.rid: r for r in _server(be, clk, 10**9).run(reqs)}
    assert res[1].admitted_s >= 5.0
    # the server was idle in between: request 0 finished long before
    assert res[0].done_s < 1.0


def test_budget_holds_requests_in_queue():
    clk = VClock()
    be = FakeBackend(clk, bytes_per_cell=1000)
    # each case needs 1 MB, the budget holds two
    reqs = [Request(i, 0.0, _spec(1000), 10) for i in range(6)]
    res = _server(be, clk, 2_000_000, slots=32, group=8, chunk=10).run(reqs)
    assert len(res) == 6
    assert be.max_resident_bytes <= 2_000_000
    assert be.max_resident_cases == 2
    # later requests waited for memory to free up
    adm = sorted(r.admitted_s for r in res)
    assert adm[2] > adm[0]


def test_request_larger_than_budget_is_rejected_and_others_served():
    """An oversized request comes back at once with FVM_ENOMEM; the requests
    around it are served, and the budget never counts it."""
    clk = VClock()
    be = FakeBackend(clk, bytes_per_cell=1000)
    reqs = [Request(0, 0.0, _spec(5), 3), Request(1, 0.0, _spec(1000), 1), Request(2, 0.0, _spec(8), 3)]
    srv = _server(be, clk, 10_000)
    res = {r.rid: r for r in srv.run(reqs)}
    assert res[1].status == -2 and res[1].bytes == 0
    assert res[0].status == 0 and res[2].status == 0
    assert be.max_resident_bytes <= 10_000 and not be.resident
    assert [rid for rid, _ in srv.rejections] == [1]


class _FailingBackend(FakeBackend):
    """footprint() raises for one request (an invalid mesh), create() for
    another (a hierarchy that cannot be built)."""

    def __init__(self, clock, bad_foot, bad_create):
        super().__init__(clock)
        self.bad_foot, self.bad_create = bad_foot, bad_create

    def footprint(self, spec):
        if getattr(spec, "rid", None) == self.bad_foot:
            raise RuntimeError("invalid mesh")
        return super().footprint(spec)

    def create(self, spec):
        if getattr(spec, "rid", None) == self.bad_create:
            raise RuntimeError("coarsening stalled")
        return super().create(spec)


def test_errors_of_one_request_do_not_stop_the_server():
    clk = VClock()
    be = _FailingBackend(clk, bad_foot=1, bad_create=3)
    reqs = [Request(i, 0.001 * i, _spec(100, rid=i), 4) for i in range(5)]
    res = {r.rid: r for r in _server(be, clk, 10**9, slots=2, group=2, chunk=2).run(reqs)}
    assert sorted(res) == [0, 1, 2, 3, 4]
    assert res[1].status == -1 and res[3].status == -1
    for i in (0, 2, 4):
        assert res[i].status == 0 and res[i].p_iters == 5 * 4
    assert not be.resident
    assert summarize(list(res.values()))["failed"] == 2


def test_slots_limit_resident_cases():
    clk = VClock()
    be = FakeBackend(clk)
    reqs = [Request(i, 0.0, _spec(100), 4) for i in range(10)]
    _server(be, clk, 10**9, slots=3, group=3, chunk=2).run(reqs)
    assert be.max_resident_cases == 3
    assert all(g[1] <= 3 for g in be.groups)


def test_continuous_batching_admits_while_others_run():
    clk = VClock()
    be = FakeBackend(clk, step_cost=1e-2)
    # a long request first, then short ones arriving while it runs
    reqs = [Request(0, 0.0, _spec(100), 100)] + [Request(i, 0.05 * i, _spec(100), 5) for i in range(1, 5)]
    res = {r.rid: r for r in _server(be, clk, 10**9, slots=8, group=8, chunk=5).run(reqs)}
    for i in range(1, 5):
        # admitted before the long request finished, and finished before it
        assert res[i].admitted_s < res[0].done_s
        assert res[i].done_s < res[0].done_s
    # shared launches: some group held more than one case
    assert max(g[1] for g in be.groups) > 1


def test_round_robin_serves_every_resident_case():
    clk = VClock()
    be = FakeBackend(clk)
    reqs = [Request(i, 0.0, _spec(100), 6) for i in range(6)]
    res = _server(be, clk, 10**9, slots=6, group=2, chunk=2).run(reqs)
    # with groups of 2 over 6 resident cases, completion is interleaved,
    # not one case after another: the first completion comes after at least
    # one advance of every other pair
    first_done = min(r.done_s for r in res)
    assert first_done >= 3 * 2 * be.step_cost


def test_failed_case_is_reported_and_released():
    clk = VClock()
    be = FakeBackend(clk, fail_rid=1)
    reqs = [Request(i, 0.0, _spec(100, rid=i), 10) for i in range(3)]
    res = {r.rid: r for r in _server(be, clk, 10**9, chunk=2).run(reqs)}
    assert res[1].status < 0
    assert res[0].status == 0 and res[2].status == 0
    assert not be.resident
    assert summarize(list(res.values()))["failed"] == 1


def test_bad_server_parameters():
    clk = VClock()
    with pytest.raises(ValueError):
        _server(FakeBackend(clk), clk, 10, slots=0)


def test_stream_ending_with_a_rejected_request():
    clk = VClock()
    be = FakeBackend(clk, bytes_per_cell=1000)
    res = _server(be, clk, 10_000).run([Request(0, 0.0, _spec(5), 2), Request(1, 0.5, _spec(1000), 1)])
    assert sorted((r.rid, r.status) for r in res) == [(0, 0), (1, -2)]


# ---------------------------------------------------------------- lanes

import threading  # noqa: E402
import time  # noqa: E402


class LaneBackend:
    """Two lanes ('small' below 500 cells, 'large' otherwise) advanced by
    separate threads in real time; an advance sleeps `cost` seconds per
    step.  Records residency and which lanes overlapped in time."""

    LANES = {"small": (4, 3), "large": (2, 2)}

    def __init__(self, cost=2e-3, bytes_per_cell=100, fail_rid=None, raise_rid=None):
        self.cost, self.bpc, self.fail_rid, self.raise_rid = cost, bytes_per_cell, fail_rid, raise_rid
        self.mu = threading.Lock()
        self.resident = {}
        self.max_bytes = 0
        self.running = {"small": 0, "large": 0}
        self.overlap = False
        self.groups = []

    def lane_of(self, spec):
        return "small" if spec.mesh.n_cells < 500 else "large"

    def footprint(self, spec):
        return spec.mesh.n_cells * self.bpc

    def create(self, spec):
        case = object()
        with self.mu:
            self.resident[id(case)] = (self.footprint(spec), spec)
            self.max_bytes = max(self.max_bytes, sum(b for b, _ in self.resident.values()))
        return case

    def advance(self, cases, n_steps, lane):
        with self.mu:
            self.running[lane] += 1
            self.overlap = self.overlap or all(v > 0 for v in self.running.values())
            self.groups.append((lane, len(cases), n_steps))
            specs = [self.resident[id(c)][1] for c in cases]
        if any(getattr(s, "rid", None) == self.raise_rid for s in specs):
            raise RuntimeError("device error")
        time.sleep(self.cost * n_steps)
        with self.mu:
            self.running[lane] -= 1
        return [{"p": [{"iters": 3}] * n_steps,
                 "status": -3 if getattr(s, "rid", None) == self.fail_rid else 0} for s in specs]

    def finish(self, case):
        with self.mu:
            del self.resident[id(case)]
        return None


def test_lanes_overlap_and_every_request_completes():
    be = LaneBackend()
    reqs = [Request(0, 0.0, _spec(2000, rid=0), 30)]
    reqs += [Request(i, 0.005 * i, _spec(100 + i, rid=i), 6) for i in range(1, 9)]
    reqs += [Request(9, 0.01, _spec(3000, rid=9), 8)]
    res = {r.rid: r for r in Server(be, 10**9, slots=8).run(reqs)}
    assert sorted(res) == list(range(10))
    assert all(r.status == 0 for r in res.values())
    assert be.overlap                       # both lanes had work on the device at once
    # the small cases did not wait for the long large one
    assert max(res[i].done_s for i in range(1, 9)) < res[0].done_s
    assert {g[0] for g in be.groups} == {"small", "large"}
    assert all(g[1] <= 4 and g[2] <= 3 for g in be.groups if g[0] == "small")
    assert all(g[1] <= 2 and g[2] <= 2 for g in be.groups if g[0] == "large")
    assert not be.resident
    assert res[3].p_iters == 3 * 6


def test_lanes_budget_rejections_and_failures():
    be = LaneBackend(bytes_per_cell=1000, fail_rid=2)
    reqs = [Request(i, 0.0, _spec(n, rid=i), 4) for i, n in enumerate([100, 200, 300, 5000, 150, 400])]
    srv = Server(be, 700_000, slots=8)
    res = {r.rid: r for r in srv.run(reqs)}
    assert sorted(res) == list(range(6))
    assert res[3].status == -2 and res[3].bytes == 0      # larger than the whole budget
    assert res[2].status == -3                            # failed on the device, released
    assert all(res[i].status == 0 for i in (0, 1, 4, 5))
    assert be.max_bytes <= 700_000 and not be.resident


def test_lanes_device_error_is_raised():
    be = LaneBackend(raise_rid=1)
    reqs = [Request(i, 0.0, _spec(100, rid=i), 3) for i in range(3)]
    with pytest.raises(RuntimeError, match="device error"):
        Server(be, 10**9).run(reqs)
