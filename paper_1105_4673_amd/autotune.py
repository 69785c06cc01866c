"""Autotuner for result-neutral launch knobs of the batched sweep.

Only knobs that cannot change a single bit of any result are tuned: waves
(blocks) per workgroup, and how many windows run per launch (one packed
launch per window, or K windows per persistent launch whose waves take work
items from a device counter).  The block edge changes the decomposition and
hence the trajectory: it is chosen per lattice-size class before any job
of the class is created (`tune_block_edges`), each candidate being a valid
decomposition of the same model, and is never changed during a run.
"""
import time

from . import fskmc as F


def _time_windows(ctx, handles, windows, reps):
    F.fskmc_sync(ctx)
    t0 = time.perf_counter()
    for _ in range(reps):
        F.fskmc_batch_advance(ctx, handles, windows)
    F.fskmc_sync(ctx)
    return (time.perf_counter() - t0) / (reps * windows)


def tune_waves_per_group(ctx, make_sims, candidates=(1, 2, 4, 8), windows=4, reps=2):
    """Time a few batched windows of freshly made sims for each candidate and
    return (best, {candidate: seconds per window}).  make_sims() must return
    new Sim objects (their state is consumed by the timing run)."""
    timings = {}
    for wpg in candidates:
        sims = make_sims()
        handles = [s.handle for s in sims]
        F.fskmc_ctx_set_waves_per_group(ctx, wpg)
        _time_windows(ctx, handles, 1, 1)  # warm-up: first use of this variant
        timings[wpg] = _time_windows(ctx, handles, windows, reps)
        for s in sims:
            s.close()
    best = min(timings, key=timings.get)
    F.fskmc_ctx_set_waves_per_group(ctx, best)
    return best, timings


def tune_windows_per_launch(ctx, make_sims, candidates=(0, 10, 50), windows=50, reps=1):
    """Time `windows` batched windows of freshly made sims per candidate
    number of windows per persistent launch (0 = one packed launch per
    window) and keep the fastest; returns (best, {candidate: seconds per
    window})."""
    timings = {}
    for k in candidates:
        sims = make_sims()
        handles = [s.handle for s in sims]
        F.fskmc_ctx_set_batch_persistent(ctx, k)
        _time_windows(ctx, handles, 1, 1)  # warm-up: first use of this variant and its graph
        timings[k] = _time_windows(ctx, handles, windows, reps)
        for s in sims:
            s.close()
    best = min(timings, key=timings.get)
    F.fskmc_ctx_set_batch_persistent(ctx, best)
    return best, timings


def _events_per_s(ctx, sims, windows):
    handles = [x.handle for x in sims]
    F.fskmc_batch_advance(ctx, handles, 1)  # warm-up: first use of the variants
    F.fskmc_sync(ctx)
    ev0 = sum(x.observe()["events"] for x in sims)
    t0 = time.perf_counter()
    F.fskmc_batch_advance(ctx, handles, windows)
    F.fskmc_sync(ctx)
    el = time.perf_counter() - t0
    return (sum(x.observe()["events"] for x in sims) - ev0) / el


def tune_block_edges(ctx, jobs, make_sim, candidates=(8, 16, 32), class_sample=16, sample=96, windows=20):
    """Block edge per lattice-size class (jobs of one (Lx, Ly)).  First each
    class alone: up to `class_sample` of its jobs with every candidate edge
    that tiles it, scored by events per second.  Then whole assignments on a
    mixed sample of up to `sample` jobs: each candidate edge for every class
    (when it tiles them all), and the per-class winners.  The batch groups
    jobs by kernel variant and launches the groups one after another, so
    mixing edges has a cost the per-class scores cannot see.  Returns the
    best assignment {(Lx, Ly): edge} and the scores {"per_class": {(Lx, Ly):
    {edge: events/s}}, "assignments": {name: events/s}, "chosen": name}.
    make_sim(job, b) must return a fresh, initialised Sim."""
    classes = {}
    for j in jobs:
        classes.setdefault((j["Lx"], j["Ly"]), []).append(j)
    tiles = lambda key, b: key[0] % (2 * b) == 0 and key[1] % (2 * b) == 0  # even blocks per row and column
    per_class = {}
    for key, members in sorted(classes.items()):
        per_class[key] = {}
        for b in candidates:
            if tiles(key, b):
                sims = [make_sim(j, b) for j in members[:class_sample]]
                per_class[key][b] = _events_per_s(ctx, sims, windows)
                for x in sims:
                    x.close()
    assignments = {"per-class": {k: max(r, key=r.get) for k, r in per_class.items()}}
    for b in candidates:
        if all(tiles(k, b) for k in classes):
            assignments[f"all-b{b}"] = {k: b for k in classes}
    mixed = jobs[:sample]
    scores = {}
    for name, assign in assignments.items():
        sims = [make_sim(j, assign[(j["Lx"], j["Ly"])]) for j in mixed]
        scores[name] = _events_per_s(ctx, sims, windows)
        for x in sims:
            x.close()
    best = max(scores, key=scores.get)
    return assignments[best], {"per_class": per_class, "assignments": scores, "chosen": best}
