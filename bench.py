#!/usr/bin/env python3
"""Benchmark of the fractional-step lattice KMC sweep on one MI355X.

Metric: KMC events per second (accepted lattice updates) on one GPU, at
bit-exact agreement with the CPU oracle (the parity tests check the same
kernels and launch configuration).

Headline (value): one timed step = one whole run of the 1024^2 Ising-type
lattice (spin flip, Arrhenius rates, J=1, h=0, beta=1, 16x16 blocks, 2 colours,
Lie dt=0.1, T=100 = 2000 windows) from a Bernoulli(1/2) start: the init kernel,
the sweep (by default all 2000 windows in one resident persistent launch:
blocks stay in LDS, neighbours exchange tagged boundary words) and the final
observables.  Each step uses its own Philox replica key.  Lattices and tables
are resident in HBM before the timed region starts.

Also in the JSON line:
  roofline      the sweep kernel's algorithmic HBM bytes per launch over its
                average launch duration (kernel-side HIP events on the launch
                stream, every k-th timed launch), against the 8 TB/s HBM peak;
  per_window    the same workload with one sweep launch per window;
  cpu_baseline  the oracle (plain single-threaded C, the blockwise scheme) on
                a bounded sample of the same workload, on this host;
  batched       512 independent Ising replicas of mixed sizes (edges
                128..1024) advanced together (one packed launch per window or
                K windows per persistent launch, both autotuned with the waves
                per workgroup), against the same 512 runs advanced one after
                another, bit-identity checked;
  served        Poisson request streams (50, 200, 1000 jobs/s) of mixed Ising
                and A/B reaction jobs (edges log-uniform in [64, 2048], T in
                [10, 200]) served with continuous batching: p50/p99
                time-to-result and aggregate events/s;
  sweep         events/s of the other (J, dt, split) points of the 1024^2
                workload (fewer steps);
  balance       workload rebalancing (Sec. 5) on a half-filled 2048^2
                lattice: one launch per window, resident launches on fixed
                block ranges and on ranges rebalanced from the previous
                launch's workload histogram, bit-identity checked;
  nested        the nested decomposition (Sec. 6) of the 1024^2 lattice
                (coarse cells of 2x2 blocks, outer Lie dt=0.1, inner Lie
                dtau=0.05): one resident launch (a workgroup per coarse cell
                for the whole run, tagged ring exchange between outer
                windows), one launch per outer window, and the flat sweeps
                (one launch per window, one persistent launch) on the same
                window list, bit-identity checked.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "KMC events/sec on 1 MI355X (plain vs batched/served) at bit-exact oracle match"
HBM_PEAK_GBS = 8000.0
LDS_PEAK_GBS = 128 * 256 * 2.4  # 128 B/clk per CU, 256 CUs, 2.4 GHz = 78.6 TB/s
# VALU issue: 256 CUs x 4 SIMDs x 2.4e9 cycles/s, one wave64 instruction per 4 cycles per SIMD
VALU_PEAK_GINST = 256 * 4 * 2.4 / 4


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def hbm_bytes(kind, b, block_windows, writes):
    """Algorithmic HBM bytes of the sweep: per block-window the block and its
    one-site halo are read (b^2 + 4b bytes) and its 16-byte counter record is
    updated (28 bytes moved: W written, two counters read and written); a block
    that changed is written back (b^2 bytes; the pair model also writes its
    halo, b^2 + 4b)."""
    rd = b * b + 4 * b
    wr = b * b if kind == "flip" else b * b + 4 * b
    return block_windows * (rd + 28) + writes * wr


def make_sim(F, ctx, wl, replica=None):
    return F.Sim(ctx, wl["kind"], wl["Lx"], wl["Ly"], wl["params"], b=wl["b"], n_colours=wl["n_colours"],
                 dt=wl["dt"], T=wl["T"], split=wl["split"], seed=wl.get("seed", 0),
                 replica=wl.get("replica", 0) if replica is None else replica)


def init_sim(sim, wl):
    sim.init(1 if wl["init"] == "bernoulli" else 0, 0.5)


def run_once(F, sim, wl):
    init_sim(sim, wl)
    sim.run_to_end()
    return sim.observe()


def resident_bytes(b, block_windows, sites, launches):
    """Algorithmic HBM bytes of the resident sweep on a square lattice of
    b x b blocks: each launch reads and writes its lattice of `sites` bytes
    once and updates each block's 16-byte counter record once (28 bytes moved:
    W written, two counters read and written); per block-window four 8-byte
    edge words are read and four written."""
    blocks = sites // (b * b)
    return launches * (2 * sites + 28 * blocks) + block_windows * 64


def lds_bytes(kind, b, block_windows, events, resident=False):
    """Algorithmic LDS bytes of the method with the block's sum tree in LDS:
    per block-window the staged block and halo (the halo only when the
    blocks stay resident), the leaves written (8n) and the n-1 inner nodes
    built from two children each (24 bytes); per accepted event a descent
    reading both children on log2 n levels (16 log2 n) and the dirty paths,
    bounded by 5 leaves (spin flip: the site and its four neighbours) or 8
    (pair events) of 8 + 24 log2 n bytes each.  The kernels here keep the
    tree in registers, so this is the method's figure, not the traffic."""
    import math
    n = b * b
    lg = math.log2(n)
    stage = 4 * b if resident else n + 4 * b
    dirty = 5 if kind == "flip" else 8
    return block_windows * (stage + 8 * n + 24 * (n - 1)) + events * (16 * lg + dirty * (8 + 24 * lg))


def nested_bytes(b, c, cells_per_launch, block_windows, launches):
    """Algorithmic HBM bytes of the nested sweep (spin flip): per launch every
    coarse cell of the active outer colour reads its c b x c b sites and the
    one-site ring around them (without corners) once and writes its sites back
    once; per block-window the 16-byte counter record is updated (28 bytes)."""
    side = c * b
    return launches * cells_per_launch * ((side + 2) ** 2 - 4 + side * side) + block_windows * 28


def measured_valu(symbol):
    """VALU wave-instructions per launch of `symbol` (rocprofv3 SQ_INSTS_VALU,
    recorded in profiles/valu.json for the workload the bench runs), or None
    when there is no record or the kernel source has changed since."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "valu.json")) as f:
            rec = json.load(f)["kernels"].get(symbol)
        with open(os.path.join(ROOT, "paper_1105_4673_amd", "csrc", "fskmc_kernels.hip"), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError, KeyError):
        return None, None
    if not rec or rec.get("kernel_source_sha256") != sha:
        return None, None
    return rec["valu_per_dispatch"], rec["source"]


def measured_traffic(symbol):
    """HBM bytes per launch of `symbol` from the rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes recorded in profiles/hbm_traffic.json (scaled by the
    copy calibration), or None when there is no record or the kernel source
    has changed since the counters were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as f:
            rec = json.load(f)["kernels"].get(symbol)
        with open(os.path.join(ROOT, "paper_1105_4673_amd", "csrc", "fskmc_kernels.hip"), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError, KeyError):
        return None, None
    if not rec or rec.get("kernel_source_sha256") != sha:
        return None, None
    return rec["traffic_bytes_per_launch"], rec["source"]


def roofline(F, ctx, kind, b, obs_list, launches, kernel_name, resident_sites=0, symbol=None):
    """Achieved algorithmic HBM GB/s of the sweep kernel: bytes per launch
    (from the run's block-window and write-back counts) over the average
    duration of the launches bracketed by kernel-side timing events."""
    ms_total, n_timed = F.fskmc_ctx_read_kernel_timing(ctx)
    bw = sum(o["block_windows"] for o in obs_list)
    wr = sum(o["writes"] for o in obs_list)
    if resident_sites:
        bytes_per_launch = resident_bytes(b, bw, resident_sites, launches) / max(launches, 1)
    elif isinstance(b, (list, tuple)):  # one block edge per simulation
        total = sum(hbm_bytes(kind, bb, o["block_windows"], o["writes"]) for bb, o in zip(b, obs_list))
        bytes_per_launch = total / max(launches, 1)
    else:
        bytes_per_launch = hbm_bytes(kind, b, bw, wr) / max(launches, 1)
    avg = ms_total / 1e3 / max(n_timed, 1)
    achieved = bytes_per_launch / avg / 1e9 if n_timed else 0.0
    traffic, source = measured_traffic(symbol)
    ev = sum(o["events"] for o in obs_list)
    if isinstance(b, (list, tuple)):
        lds = sum(lds_bytes(kind, bb, o["block_windows"], o["events"]) for bb, o in zip(b, obs_list))
    else:
        lds = lds_bytes(kind, b, bw, ev, resident=bool(resident_sites))
    lds_per_launch = lds / max(launches, 1)
    lds_achieved = lds_per_launch / avg / 1e9 if n_timed else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": source, "kernel": kernel_name,
            "bytes_per_launch": bytes_per_launch, "avg_launch_us": avg * 1e6, "timed_launches": n_timed,
            "lds": {"bound": "lds", "achieved": lds_achieved, "peak": LDS_PEAK_GBS, "unit": "GB/s",
                    "frac": lds_achieved / LDS_PEAK_GBS, "bytes_per_launch": lds_per_launch},
            "alu": alu_term(symbol, avg if n_timed else 0.0)}


def alu_term(symbol, avg_s):
    """Measured VALU issue rate of a launch against the chip's issue peak
    (recorded SQ_INSTS_VALU per launch over the measured launch duration): a
    utilisation of the SIMDs, not an algorithmic operation count."""
    valu, source = measured_valu(symbol) if symbol else (None, None)
    if valu is None or avg_s <= 0:
        return None
    achieved = valu / avg_s / 1e9
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_GINST, "unit": "Ginst/s",
            "frac": achieved / VALU_PEAK_GINST, "valu_per_launch": valu, "valu_source": source}


def bench_plain(F, ctx, wl, steps, warmup, stride, persist=0, resident=False, wpg=2):
    sims = [make_sim(F, ctx, wl, replica=i) for i in range(warmup + steps)]
    for i in range(warmup):
        run_once(F, sims[i], wl)
    F.fskmc_sync(ctx)
    F.fskmc_ctx_read_kernel_timing(ctx)  # discard
    F.fskmc_ctx_set_kernel_timing(ctx, stride)
    F.fskmc_sync(ctx)
    t0 = time.perf_counter()
    obs = [run_once(F, sims[warmup + i], wl) for i in range(steps)]
    F.fskmc_sync(ctx)
    el = time.perf_counter() - t0
    P = wl["b"] ** 2 // 64
    if persist > 0:
        launches = sum(-(-o["window"] // persist) for o in obs)
        kname = (f"k_sweep_{'resident' if resident else 'persistent'}<P={P},{wl['kind']}> "
                 f"({persist} windows per launch)")
        cap = 4 if P == 16 else 8  # blocks a resident wave can hold
        symbol = f"k_sweep_resident<{P}, {wl['b']}, {wl['b']}, {1 if wpg == 1 else 2}, {cap}>" if resident else None
    else:
        launches = sum(o["window"] for o in obs)
        kname = f"k_sweep_single<P={P},{wl['kind']}>"
        symbol = f"k_sweep_single<{P}, {wl['b']}, {wl['b']}, {1 if wl['kind'] == 'flip' else 2}, {wpg}>"
    rl = roofline(F, ctx, wl["kind"], wl["b"], obs, launches, kname,
                  resident_sites=wl["Lx"] * wl["Ly"] if resident else 0, symbol=symbol)
    F.fskmc_ctx_set_kernel_timing(ctx, 0)
    for s in sims:
        s.close()
    events = sum(o["events"] for o in obs)
    return {"events": events, "seconds": el, "obs": obs, "roofline": rl,
            "windows": sum(o["window"] for o in obs)}


def cpu_baseline(wl, seconds):
    """Oracle events/s on a bounded sample: consecutive windows of replica 0
    from the workload's own initial state, until `seconds` of CPU time."""
    import numpy as np
    import oracle
    if wl["kind"] == "flip":
        k_a, k_d, J, h, beta = wl["params"]
        model = oracle.Model("flip", wl["Lx"], wl["Ly"], k_a=k_a, k_d=k_d, J=J, h=h, beta=beta)
    else:
        y, k_r, D = wl["params"]
        model = oracle.Model("zgb", wl["Lx"], wl["Ly"], y=y, k_r=k_r, D=D)
    b = wl["b"]
    cmap = oracle.colour_map(model, b, b, wl["n_colours"])
    cols, durs, _ = oracle.schedule(wl["split"], wl["n_colours"], wl["dt"], wl["T"])
    lat = oracle.init_bernoulli(model.N, 0.5, 0, 0) if wl["init"] == "bernoulli" else np.zeros(model.N, np.uint8)
    t0 = time.process_time()
    w = events = 0
    while w < len(cols) and time.process_time() - t0 < seconds:
        n = min(2, len(cols) - w)
        res = oracle.fs_run(model, lat, b, b, cmap, wl["n_colours"], cols[w:w + n], durs[w:w + n], 0, 0, w0=w)
        lat = res["lattice"]
        events += res["events"]
        w += n
    el = time.process_time() - t0
    return {"value": events / el, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"{wl['name']}: windows [0,{w}) of {len(cols)} of replica 0 from the same start, "
                      f"single-threaded, {events} events in {el:.1f} s CPU"}


def bench_batched(F, ctx, n_jobs, stride, chunk=50, wpg=0, k=-1, sequential=True, block_edge=0):
    """512 (n_jobs) Ising replicas in one packed launch per window vs the same
    replicas advanced one at a time; every job's final lattice compared."""
    import hashlib
    from paper_1105_4673_amd import autotune, workloads
    jobs = workloads.c3_jobs(n=n_jobs)

    def make_all(sel):
        out = []
        for j in sel:
            s = make_sim(F, ctx, j)
            init_sim(s, j)
            out.append(s)
        return out

    def make_b(j, b):
        s = make_sim(F, ctx, dict(j, b=b))
        init_sim(s, j)
        return s

    if block_edge:
        edges = {(j["Lx"], j["Ly"]): block_edge for j in jobs}
        edge_rates = {"chosen": f"all-b{block_edge} (fixed)", "assignments": None, "per_class": None}
    else:
        edges, edge_rates = autotune.tune_block_edges(ctx, jobs, make_b)
    log(f"block edge per size: {edges}")
    jobs = [dict(j, b=edges[(j["Lx"], j["Ly"])]) for j in jobs]
    if wpg:
        best, timings = wpg, None
        F.fskmc_ctx_set_waves_per_group(ctx, wpg)
    else:
        best, timings = autotune.tune_waves_per_group(ctx, lambda: make_all(jobs[:96]))
    log(f"waves/group: {best} {timings}")
    if k >= 0:
        best_k, timings_k = k, None
        F.fskmc_ctx_set_batch_persistent(ctx, k)
    else:
        best_k, timings_k = autotune.tune_windows_per_launch(ctx, lambda: make_all(jobs[:96]))
    log(f"windows per launch: {best_k} {timings_k}")
    sims = make_all(jobs)
    handles = [s.handle for s in sims]
    F.fskmc_sync(ctx)
    F.fskmc_ctx_read_kernel_timing(ctx)
    F.fskmc_ctx_set_kernel_timing(ctx, stride)
    launches = 0
    t0 = time.perf_counter()
    while True:
        left = max(s.windows()[0] - s.windows()[1] for s in sims)
        if left == 0:
            break
        F.fskmc_batch_advance(ctx, handles, min(chunk, left))
        launches += min(chunk, left)
    F.fskmc_sync(ctx)
    el = time.perf_counter() - t0
    obs = [s.observe() for s in sims]
    if best_k:
        launches = -(-launches // best_k)
    P = jobs[0]["b"] ** 2 // 64
    symbol = None if best_k or any(j["b"] != jobs[0]["b"] for j in jobs) else \
        f"k_sweep_batched<{P}, {jobs[0]['b']}, {jobs[0]['b']}, 1, {best}>"
    rl = roofline(F, ctx, "flip", [j["b"] for j in jobs], obs, launches,
                  "k_sweep_batched_persistent<P=4,flip>" if best_k else "k_sweep_batched<P=4,flip>", symbol=symbol)
    F.fskmc_ctx_set_kernel_timing(ctx, 0)
    F.fskmc_ctx_set_batch_persistent(ctx, 0)
    ev_b = sum(o["events"] for o in obs)
    dig_b = [hashlib.sha256(s.lattice().tobytes()).hexdigest() for s in sims]
    for s in sims:
        s.close()
    log(f"batched: {ev_b} events in {el:.3f} s")

    if sequential:
        seq = make_all(jobs)
        F.fskmc_sync(ctx)
        t0 = time.perf_counter()
        for s in seq:
            s.run_to_end()
        F.fskmc_sync(ctx)
        el_s = time.perf_counter() - t0
        obs_s = [s.observe() for s in seq]
        ev_s = sum(o["events"] for o in obs_s)
        dig_s = [hashlib.sha256(s.lattice().tobytes()).hexdigest() for s in seq]
        for s in seq:
            s.close()
        log(f"sequential: {ev_s} events in {el_s:.3f} s")
        identical = dig_b == dig_s and ev_b == ev_s
    else:  # counter runs: the 10^5 sequential launches are not needed
        el_s, ev_s, identical = None, None, None
    sites = sum(j["Lx"] * j["Ly"] for j in jobs)
    bname = "b16" if all(j["b"] == 16 for j in jobs) else "bauto"
    return {"workload": f"ising_x{n_jobs}_edges128-1024_{bname}_lie_dt0.1_T10", "jobs": n_jobs, "sites": sites,
            "value": ev_b / el, "unit": "events/s", "seconds": el, "events": ev_b,
            "sequential_value": ev_s / el_s if sequential else None, "sequential_seconds": el_s if sequential else None,
            "speedup_vs_sequential": (ev_b / el) / (ev_s / el_s) if sequential else None,
            "bit_identical_to_sequential": identical,
            "block_edge_by_size": {f"{k[0]}x{k[1]}": v for k, v in edges.items()},
            "autotune_block_edge": {"chosen": edge_rates["chosen"], "assignments_events_per_s": edge_rates["assignments"],
                                    "per_class_events_per_s": None if edge_rates["per_class"] is None else
                                    {f"{k[0]}x{k[1]}": r for k, r in edge_rates["per_class"].items()}},
            "waves_per_group": best, "autotune_s_per_window": timings, "windows_per_launch": best_k,
            "autotune_windows_per_launch_s_per_window": timings_k, "roofline": rl}


def bench_balance(F, ctx, windows, chunk):
    """Workload rebalancing (Sec. 5) on the half-filled 2048^2 lattice: the
    first `windows` windows with one launch per window, with resident launches
    of `chunk` windows on fixed block ranges, and on ranges rebalanced from the
    previous launch's workload; final lattices compared."""
    import hashlib
    import numpy as np
    from paper_1105_4673_amd import workloads
    wl = workloads.half_filled()
    N = wl["Lx"] * wl["Ly"]
    lat0 = np.zeros(N, np.uint8)
    lat0[N // 2:] = 1
    out = {"workload": wl["name"], "windows": windows, "windows_per_launch": chunk}
    digests = []
    for label, persist, rebalance in (("per_window", 0, 0), ("resident_fixed", chunk, 0),
                                      ("resident_rebalanced", chunk, 1)):
        F.fskmc_ctx_set_persistent(ctx, persist)
        F.fskmc_ctx_set_rebalance(ctx, rebalance)
        best = None
        for rep in range(2):  # the first pass also warms the kernels up
            s = make_sim(F, ctx, wl, replica=3)
            s.set_lattice(lat0)
            F.fskmc_sync(ctx)
            t0 = time.perf_counter()
            s.advance(windows)
            F.fskmc_sync(ctx)
            el = time.perf_counter() - t0
            ev = s.observe()["events"]
            dig = hashlib.sha256(s.lattice().tobytes()).hexdigest()
            s.close()
            best = el if best is None else min(best, el)
        out[label] = {"value": ev / best, "seconds": best, "events": ev}
        digests.append(dig)
        log(f"balance {label}: {ev / best:.3g} events/s")
    F.fskmc_ctx_set_rebalance(ctx, 0)
    F.fskmc_ctx_set_persistent(ctx, 0)
    out["bit_identical"] = len(set(digests)) == 1
    out["speedup_rebalanced_vs_fixed"] = out["resident_rebalanced"]["value"] / out["resident_fixed"]["value"]
    return out


def bench_nested(F, ctx, T, dtau, c, stride):
    """Nested decomposition (Sec. 6) of the 1024^2 lattice, whole runs to T:
    the nested kernel (one launch per outer window), the flat per-window
    sweep and the flat persistent sweep on the same window list."""
    import hashlib
    from paper_1105_4673_amd import workloads
    wl = workloads.nested(c=c, dtau=dtau, T=T)
    out = {"workload": wl["name"]}
    digests = []
    for label, knob, persist in (("nested_resident", 1, 100000), ("nested_kernel", 1, 0), ("flat_per_window", 0, 0),
                                 ("flat_persistent", 0, 100000)):
        F.fskmc_ctx_set_nested(ctx, knob)
        F.fskmc_ctx_set_persistent(ctx, persist)
        best = None
        for rep in range(2):  # the first pass also warms the kernels up
            s = F.Sim(ctx, wl["kind"], wl["Lx"], wl["Ly"], wl["params"], b=wl["b"], dt=wl["dt"], T=wl["T"],
                      split=wl["split"], seed=0, replica=11, nested=wl["nested"])
            init_sim(s, wl)
            F.fskmc_sync(ctx)
            if knob:
                F.fskmc_ctx_read_kernel_timing(ctx)  # discard
                F.fskmc_ctx_set_kernel_timing(ctx, stride)
            t0 = time.perf_counter()
            s.run_to_end()
            F.fskmc_sync(ctx)
            el = time.perf_counter() - t0
            if knob:
                kms, kn = F.fskmc_ctx_read_kernel_timing(ctx)
                F.fskmc_ctx_set_kernel_timing(ctx, 0)
            obs = s.observe()
            dig = hashlib.sha256(s.lattice().tobytes()).hexdigest()
            windows = s.windows()[0]
            s.close()
            if best is None or el < best[0]:
                best = (el, obs, (kms, kn) if knob else None)
        el, obs, timing = best
        ev = obs["events"]
        out[label] = {"value": ev / el, "seconds": el, "events": ev}
        if timing is not None and not persist:
            # outer windows = launches: the outer Lie scheme has 2 per step
            launches = int(round(wl["T"] / wl["dt"])) * 2
            cells = (wl["Lx"] // (c * wl["b"])) * (wl["Ly"] // (c * wl["b"])) // 2
            per_launch = nested_bytes(wl["b"], c, cells, obs["block_windows"], launches) / launches
            avg = timing[0] / 1e3 / max(timing[1], 1)
            achieved = per_launch / avg / 1e9
            P = wl["b"] ** 2 // 64
            traffic, source = measured_traffic(f"k_sweep_nested<{P}, {wl['b']}, 1, {c}, 2>")
            out[label]["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                      "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                                      "traffic_source": source, "kernel": f"k_sweep_nested<P={P},c={c}>",
                                      "bytes_per_launch": per_launch, "avg_launch_us": avg * 1e6,
                                      "timed_launches": timing[1], "launches": launches}
        digests.append(dig)
        log(f"nested {label}: {ev / el:.3g} events/s ({el * 1e3:.1f} ms, {windows} windows)")
    F.fskmc_ctx_set_nested(ctx, 1)
    F.fskmc_ctx_set_persistent(ctx, 0)
    out["bit_identical"] = len(set(digests)) == 1
    out["speedup_vs_flat_per_window"] = out["nested_resident"]["value"] / out["flat_per_window"]["value"]
    out["speedup_vs_flat_persistent"] = out["nested_resident"]["value"] / out["flat_persistent"]["value"]
    return out


def bench_served(F, ctx, rates, n_jobs, windows_per_step, budget_gib):
    """Poisson request streams of mixed Ising / reaction jobs served with
    continuous batching; time-to-result percentiles and aggregate events/s."""
    from paper_1105_4673_amd import workloads
    from paper_1105_4673_amd.serve import GpuBackend, Request, Server, summarize
    out = []
    for rate in rates:
        reqs = [Request(i, spec, spec["arrival"]) for i, spec in enumerate(workloads.c4_requests(rate, n=n_jobs))]
        srv = Server(GpuBackend(ctx), hbm_budget=int(budget_gib * (1 << 30)), max_slots=n_jobs,
                     windows_per_step=windows_per_step)
        t0 = time.perf_counter()
        done = srv.run(reqs)
        wall = time.perf_counter() - t0
        s = summarize(done, wall)
        s.update({"rate_jobs_per_s": rate, "requests": n_jobs, "batched_steps": srv.steps,
                  "last_arrival_s": max(r.arrival for r in reqs),
                  "sites_mean": sum(r.spec["Lx"] * r.spec["Ly"] for r in reqs) / n_jobs})
        log(f"served rate {rate}/s: {s['jobs']} jobs, {s['events']} events in {wall:.2f} s, "
            f"p50 {s['p50_time_to_result_s']:.3f} s p99 {s['p99_time_to_result_s']:.3f} s")
        out.append(s)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--J", type=float, default=1.0)
    ap.add_argument("--dt", type=float, default=0.1)
    ap.add_argument("--split", type=int, default=0)
    ap.add_argument("--timing-stride", type=int, default=8,
                    help="bracket every k-th sweep launch with kernel-side HIP timing events")
    ap.add_argument("--waves-per-group", type=int, default=2)
    ap.add_argument("--persistent", type=int, default=100000,
                    help="windows per persistent launch for single-lattice runs (default: the whole run in one "
                         "launch; 0: one launch per window)")
    ap.add_argument("--no-resident", action="store_true",
                    help="persistent sweeps stream every block from HBM each window instead of keeping it in LDS")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-jobs", type=int, default=512, help="0 skips the batched measurement")
    ap.add_argument("--sweep", action="store_true", help="also time the other (J, dt, split) points")
    ap.add_argument("--served-jobs", type=int, default=64, help="requests per arrival rate; 0 skips serving")
    ap.add_argument("--served-rates", default="50,200,1000")
    ap.add_argument("--served-windows-per-step", type=int, default=4)
    ap.add_argument("--balance-windows", type=int, default=200,
                    help="windows of the half-filled 2048^2 rebalancing comparison; 0 skips it")
    ap.add_argument("--balance-chunk", type=int, default=20)
    ap.add_argument("--batched-wpg", type=int, default=0,
                    help="waves per workgroup of the batched launches (0: autotuned)")
    ap.add_argument("--batched-windows-per-launch", type=int, default=-1,
                    help="windows per batched launch (0: one packed launch per window; -1: autotuned)")
    ap.add_argument("--batched-sequential", type=int, default=1,
                    help="0 skips the sequential comparison of the batched measurement")
    ap.add_argument("--batched-block-edge", type=int, default=0,
                    help="block edge of every batched job (0: autotuned per lattice size)")
    ap.add_argument("--nested-T", type=float, default=20.0, help="0 skips the nested measurement")
    ap.add_argument("--nested-dtau", type=float, default=0.05)
    ap.add_argument("--nested-cell", type=int, default=2)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the fractional-step sweep runs on a single MI355X here)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        n = args.copy_probe << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n}), flush=True)
        return

    from paper_1105_4673_amd import fskmc as F
    from paper_1105_4673_amd import workloads

    torch.cuda.init()
    ctx = F.fskmc_ctx_create(0, torch.cuda.current_stream().cuda_stream)
    F.fskmc_ctx_set_waves_per_group(ctx, args.waves_per_group)
    F.fskmc_ctx_set_persistent(ctx, args.persistent)
    F.fskmc_ctx_set_resident(ctx, not args.no_resident)
    wl = workloads.c1(J=args.J, dt=args.dt, split=args.split)
    log(f"workload {wl['name']}")
    resident = args.persistent > 0 and not args.no_resident
    p = bench_plain(F, ctx, wl, args.steps, args.warmup, args.timing_stride, args.persistent, resident,
                    args.waves_per_group)
    log(f"plain: {args.steps} steps, {p['events']} events in {p['seconds']:.3f} s, "
        f"kernel avg {p['roofline']['avg_launch_us']:.2f} us")
    result = {
        "metric": METRIC,
        "value": p["events"] / p["seconds"],
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": p["seconds"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "lattice": [wl["Lx"], wl["Ly"]], "block": [wl["b"], wl["b"]],
                   "colours": wl["n_colours"], "windows_per_step": p["windows"] // args.steps,
                   "events_per_step": p["events"] / args.steps, "waves_per_group": args.waves_per_group,
                   "persistent_windows_per_launch": args.persistent, "resident": resident},
        "roofline": p["roofline"],
    }
    if args.persistent > 0:
        F.fskmc_ctx_set_persistent(ctx, 0)
        q = bench_plain(F, ctx, wl, min(args.steps, 3), 1, args.timing_stride, 0, wpg=args.waves_per_group)
        F.fskmc_ctx_set_persistent(ctx, args.persistent)
        result["per_window"] = {"value": q["events"] / q["seconds"], "ms_per_step": q["seconds"] * 1e3 / min(args.steps, 3),
                                "roofline": q["roofline"]}
        log(f"one launch per window: {result['per_window']['value']:.3g} events/s")
    if args.sweep:
        sweep = []
        for J in (0.5, 1.0, 2.0):
            for dt in (0.01, 0.1, 1.0):
                for split in (0, 1):
                    w2 = workloads.c1(J=J, dt=dt, split=split)
                    q = bench_plain(F, ctx, w2, 1, 1, 0, args.persistent, resident, args.waves_per_group)
                    sweep.append({"workload": w2["name"], "value": q["events"] / q["seconds"],
                                  "ms_per_step": q["seconds"] * 1e3, "events_per_step": q["events"]})
                    log(f"sweep {w2['name']}: {q['events'] / q['seconds']:.3g} events/s")
        result["sweep"] = sweep
    if args.balance_windows:
        result["balance"] = bench_balance(F, ctx, args.balance_windows, args.balance_chunk)
    if args.nested_T:
        result["nested"] = bench_nested(F, ctx, args.nested_T, args.nested_dtau, args.nested_cell,
                                        args.timing_stride)
    F.fskmc_ctx_set_persistent(ctx, 0)  # batched and served runs use one packed launch per window
    if args.batched_jobs:
        F.fskmc_ctx_set_waves_per_group(ctx, args.waves_per_group)
        result["batched"] = bench_batched(F, ctx, args.batched_jobs, args.timing_stride, wpg=args.batched_wpg,
                                          k=args.batched_windows_per_launch,
                                          sequential=bool(args.batched_sequential),
                                          block_edge=args.batched_block_edge)
    if args.served_jobs:
        F.fskmc_ctx_set_waves_per_group(ctx, args.waves_per_group)
        result["served"] = bench_served(F, ctx, [float(r) for r in args.served_rates.split(",")], args.served_jobs,
                                        args.served_windows_per_step, budget_gib=64.0)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    F.fskmc_ctx_destroy(ctx)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
