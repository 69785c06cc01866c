"""Serving loop: continuous batching of fractional-step KMC jobs on one GPU.

Requests arrive over time (e.g. a Poisson stream).  The loop admits a request
as soon as it has arrived, a slot is free and its device footprint fits the
HBM budget; every resident job keeps its lattice and window counter on the
device; each iteration advances every resident job by a few windows in one
batched launch per window (jobs of different sizes, models and schedules are
packed into the same grid); finished jobs are retired, their results read
back and their memory released, so waiting requests take their place.  A job's
result does not depend on what it was batched with: its random numbers are
keyed by (job key, block, window, draw).

The backend is injectable so the scheduling policy can be tested without a
GPU (see tests/test_serve_policy.py).
"""
import collections
import hashlib
import time


class Request:
    __slots__ = ("rid", "spec", "arrival", "admitted", "finished", "result", "handle", "footprint", "status")

    def __init__(self, rid, spec, arrival):
        self.rid = rid
        self.spec = spec
        self.arrival = arrival
        self.admitted = None
        self.finished = None
        self.result = None
        self.handle = None
        self.footprint = 0
        self.status = "queued"

    @property
    def time_to_result(self):
        return None if self.finished is None else self.finished - self.arrival


class GpuBackend:
    """libfskmc on one GPU context.

    By default the batched advances launch directly instead of replaying a
    captured graph (the context's graph knob is set accordingly): the resident
    set changes from step to step, so a graph would be captured again for
    most steps, and direct launches let the groups of different models run
    side by side on streams of their own."""

    def __init__(self, ctx, graphs=False):
        from . import fskmc
        self.F = fskmc
        self.ctx = ctx
        fskmc.fskmc_ctx_set_graphs(ctx, graphs)

    def footprint(self, spec):
        F = self.F
        model = F.FSKMC_MODEL_FLIP if spec["kind"] == "flip" else F.FSKMC_MODEL_ZGB
        return F.fskmc_sim_footprint(2, spec["Lx"], spec["Ly"], model, spec["b"], spec["b"], spec["n_colours"],
                                     spec["dt"], spec["T"], spec["split"])

    def start(self, spec):
        s = self.F.Sim(self.ctx, spec["kind"], spec["Lx"], spec["Ly"], spec["params"], b=spec["b"],
                       n_colours=spec["n_colours"], dt=spec["dt"], T=spec["T"], split=spec["split"],
                       seed=spec.get("seed", 0), replica=spec.get("replica", 0))
        s.init(1 if spec.get("init") == "bernoulli" else 0, 0.5)
        return s

    def advance(self, handles, windows):
        self.F.fskmc_batch_advance(self.ctx, [h.handle for h in handles], windows)

    def progress(self, h):
        total, nxt = h.windows()
        return nxt, total

    def finish(self, h):
        obs = h.observe()
        digest = hashlib.sha256(h.lattice().tobytes()).hexdigest()
        h.close()
        return {"events": obs["events"], "counts": obs["count"], "bonds_equal": obs["bonds_equal"],
                "bonds_ab": obs["bonds_ab"], "t": obs["t"], "digest": digest}

    def cancel(self, h):
        h.close()

    def sync(self):
        self.F.fskmc_sync(self.ctx)


class Server:
    """Admission by footprint and slots, continuous batching, retirement."""

    def __init__(self, backend, hbm_budget, max_slots=1024, windows_per_step=4, clock=time.perf_counter,
                 admit_per_step=None):
        self.b = backend
        self.budget = int(hbm_budget)
        self.max_slots = int(max_slots)
        self.k = int(windows_per_step)
        # at most this many admissions per iteration (None: all that fit), so
        # that a burst of arrivals is set up between launches of the jobs
        # already resident instead of while the GPU waits for its first launch
        self.admit_per_step = admit_per_step
        self.clock = clock
        self.queue = collections.deque()
        self.resident = []
        self.done = []
        self.rejected = []
        self.used = 0
        self.steps = 0
        self.max_resident = 0

    def submit(self, req):
        req.footprint = self.b.footprint(req.spec)
        if req.footprint <= 0 or req.footprint > self.budget:
            req.status = "rejected"  # can never fit: refuse instead of blocking the queue
            self.rejected.append(req)
            return False
        self.queue.append(req)
        return True

    def cancel(self, rid):
        for r in list(self.resident):
            if r.rid == rid:
                self.b.cancel(r.handle)
                self.resident.remove(r)
                self.used -= r.footprint
                r.status = "cancelled"
                r.finished = self.clock()
                self.done.append(r)
                return True
        for r in list(self.queue):
            if r.rid == rid:
                self.queue.remove(r)
                r.status = "cancelled"
                self.done.append(r)
                return True
        return False

    def _admit(self, now):
        # first come, first served: the head of the queue waits for room
        admitted = 0
        while self.queue and self.queue[0].arrival <= now and len(self.resident) < self.max_slots:
            if self.admit_per_step is not None and admitted >= self.admit_per_step and self.resident:
                break
            r = self.queue[0]
            if self.used + r.footprint > self.budget:
                break
            self.queue.popleft()
            r.handle = self.b.start(r.spec)
            r.admitted = now
            r.status = "running"
            self.used += r.footprint
            self.resident.append(r)
            admitted += 1

    def _retire(self):
        keep = []
        for r in self.resident:
            nxt, total = self.b.progress(r.handle)
            if nxt >= total:
                r.result = self.b.finish(r.handle)
                r.finished = self.clock()
                r.status = "done"
                self.used -= r.footprint
                self.done.append(r)
            else:
                keep.append(r)
        self.resident = keep

    def step(self):
        """One iteration: admit, one batched advance, retire.  Returns False
        when there is nothing left to do."""
        now = self.clock()
        self._admit(now)
        if self.resident:
            self.max_resident = max(self.max_resident, len(self.resident))
            self.b.advance([r.handle for r in self.resident], self.k)
            self.steps += 1
            self._retire()
            return True
        return bool(self.queue)

    def run(self, requests, idle_wait=1e-4, sleep=time.sleep):
        """Serve requests whose `arrival` times are relative to the start of
        this call; returns the finished requests in completion order."""
        t0 = self.clock()
        clock0 = self.clock
        self.clock = lambda: clock0() - t0
        try:
            for r in sorted(requests, key=lambda q: q.arrival):
                self.submit(r)
            while self.queue or self.resident:
                self.step()
                if not self.resident and self.queue:
                    wait = self.queue[0].arrival - self.clock()
                    if wait > 0:
                        sleep(min(wait, idle_wait * 100))
            return list(self.done)
        finally:
            self.clock = clock0


def percentile(values, q):
    """Nearest-rank percentile (q in [0,100]) of a non-empty list."""
    v = sorted(values)
    k = max(0, min(len(v) - 1, int(-(-q * len(v) // 100)) - 1))
    return v[k]


def summarize(done, wall):
    ok = [r for r in done if r.status == "done"]
    ttr = [r.time_to_result for r in ok]
    events = sum(r.result["events"] for r in ok)
    return {"jobs": len(ok), "events": events, "wall_s": wall, "events_per_s": events / wall if wall > 0 else 0.0,
            "p50_time_to_result_s": percentile(ttr, 50) if ttr else None,
            "p99_time_to_result_s": percentile(ttr, 99) if ttr else None}
