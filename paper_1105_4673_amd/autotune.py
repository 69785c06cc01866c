"""Autotuner for result-neutral launch knobs of the batched sweep.

Only knobs that cannot change a single bit of any result are tuned: waves
(blocks) per workgroup, and how many windows run per launch (one packed
launch per window, or K windows per persistent launch whose waves take work
items from a device counter).  The block edge changes the decomposition and
hence the trajectory, so it is fixed per job before the run and never tuned
here.
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
