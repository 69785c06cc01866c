"""Host-side tests of the serving loop's policy (no GPU): admission by arrival
time, slots and HBM footprint; continuous batching (jobs join and leave
between steps); first-come-first-served; refusal of jobs that can never fit;
cancellation; percentiles."""
from paper_1105_4673_amd.serve import Request, Server, percentile, summarize


class FakeJob:
    def __init__(self, spec):
        self.spec = spec
        self.w = 0
        self.total = spec["windows"]


class FakeBackend:
    """Each job needs spec['windows'] windows; advancing a batch costs one
    tick of a virtual clock per window."""

    def __init__(self, clock):
        self.clock = clock
        self.batches = []

    def footprint(self, spec):
        return spec["bytes"]

    def start(self, spec):
        return FakeJob(spec)

    def advance(self, handles, windows):
        self.batches.append(sorted(h.spec["name"] for h in handles))
        for h in handles:
            h.w = min(h.total, h.w + windows)
        self.clock.t += windows

    def progress(self, h):
        return h.w, h.total

    def finish(self, h):
        return {"events": h.total * 10}

    def cancel(self, h):
        pass


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def _sleep(clock):
    def s(dt):
        clock.t += dt
    return s


def _req(i, arrival, windows, nbytes):
    return Request(i, {"name": f"j{i}", "windows": windows, "bytes": nbytes}, arrival)


def test_continuous_batching_and_fifo():
    clk = Clock()
    be = FakeBackend(clk)
    srv = Server(be, hbm_budget=100, max_slots=2, windows_per_step=1, clock=clk)
    reqs = [_req(0, 0.0, 3, 10), _req(1, 0.0, 1, 10), _req(2, 0.0, 2, 10), _req(3, 5.0, 1, 10)]
    done = srv.run(reqs, sleep=_sleep(clk))
    assert [r.rid for r in done if r.status == "done"] == [1, 0, 2, 3]
    # j2 joined as soon as j1 left (slot freed), j3 only after it arrived
    assert be.batches[0] == ["j0", "j1"]
    assert be.batches[1] == ["j0", "j2"]
    assert all(r.finished >= r.arrival for r in done)
    assert srv.used == 0 and not srv.resident


def test_budget_blocks_head_and_refuses_impossible():
    clk = Clock()
    be = FakeBackend(clk)
    srv = Server(be, hbm_budget=100, max_slots=10, windows_per_step=1, clock=clk)
    reqs = [_req(0, 0.0, 4, 70), _req(1, 0.0, 1, 50), _req(2, 0.0, 1, 20), _req(3, 0.0, 1, 500)]
    done = srv.run(reqs, sleep=_sleep(clk))
    assert [r.rid for r in srv.rejected] == [3]
    # j1 does not fit beside j0; first come first served keeps j2 behind j1
    assert be.batches[0] == ["j0"]
    order = [r.rid for r in done]
    assert order.index(0) < order.index(1) < order.index(2)
    assert max(len(b) for b in be.batches) <= 2


def test_cancel_running_and_queued():
    clk = Clock()
    be = FakeBackend(clk)
    srv = Server(be, hbm_budget=100, max_slots=1, windows_per_step=1, clock=clk)
    for r in [_req(0, 0.0, 10, 10), _req(1, 0.0, 2, 10), _req(2, 0.0, 2, 10)]:
        srv.submit(r)
    srv.step()
    assert srv.cancel(0) and srv.cancel(2)
    while srv.queue or srv.resident:
        srv.step()
    st = {r.rid: r.status for r in srv.done}
    assert st == {0: "cancelled", 1: "done", 2: "cancelled"}
    assert srv.used == 0


def test_percentiles_and_summary():
    assert percentile([3, 1, 2], 50) == 2
    assert percentile(list(range(1, 101)), 99) == 99
    assert percentile([5.0], 99) == 5.0
    clk = Clock()
    be = FakeBackend(clk)
    srv = Server(be, hbm_budget=100, max_slots=4, windows_per_step=2, clock=clk)
    done = srv.run([_req(i, float(i), 3, 10) for i in range(8)], sleep=_sleep(clk))
    s = summarize(done, wall=clk.t)
    assert s["jobs"] == 8 and s["events"] == 8 * 30
    assert s["p50_time_to_result_s"] <= s["p99_time_to_result_s"]


def test_admissions_per_step_are_limited_in_arrival_order():
    """A burst of five arrivals with at most two admissions per step: two jobs
    join the first launch, two more the second, the last the third, in
    arrival order; every job still finishes."""
    clk = Clock()
    be = FakeBackend(clk)
    srv = Server(be, hbm_budget=100, max_slots=10, windows_per_step=1, clock=clk, admit_per_step=2)
    reqs = [_req(i, 0.0, 4, 10) for i in range(5)]
    done = srv.run(reqs, sleep=_sleep(clk))
    assert be.batches[0] == ["j0", "j1"]
    assert be.batches[1] == ["j0", "j1", "j2", "j3"]
    assert be.batches[2] == ["j0", "j1", "j2", "j3", "j4"]
    assert sorted(r.rid for r in done if r.status == "done") == [0, 1, 2, 3, 4]
    assert [r.admitted for r in sorted(done, key=lambda q: q.rid)] == [0.0, 0.0, 1.0, 1.0, 2.0]
