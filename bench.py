#!/usr/bin/env python3
"""Benchmark of the fractional-step lattice KMC sweep on one MI355X.

Metric: KMC events per second (accepted lattice updates) on one GPU, at
bit-exact agreement with the CPU oracle (the parity tests check the same
kernels and launch configuration).

Timed step (default workload): one whole run of the 1024^2 Ising-type lattice
(spin flip, Arrhenius rates, J=1, h=0, beta=1, 16x16 blocks, 2 colours, Lie
dt=0.1, T=100 = 2000 windows) from a Bernoulli(1/2) start: init kernel, every
window's sweep launch, and the final observables.  Each step uses its own
Philox replica key.  The lattice and all tables are resident in HBM before the
timed region starts.

The JSON line also carries:
  roofline      the sweep kernel's algorithmic HBM bytes per launch over its
                average launch duration (HIP events on the launch stream, a
                sample of the timed launches), against the 8 TB/s HBM peak;
  cpu_baseline  the oracle (plain single-threaded C, the blockwise scheme) on
                a bounded sample of the same workload, on this host.
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def hbm_bytes(kind, b, block_windows, writes):
    """Algorithmic HBM bytes of the sweep: per block-window the block and its
    one-site halo are read (b^2 + 4b bytes); a block that changed is written
    back (b^2 bytes; the pair model also writes its halo); the block's event
    counters are updated (4 + 2*8 + 2*4 bytes)."""
    rd = b * b + 4 * b
    wr = b * b if kind == "flip" else b * b + 4 * b
    return block_windows * (rd + 28) + writes * wr


def make_sim(F, ctx, wl, replica):
    s = F.Sim(ctx, wl["kind"], wl["Lx"], wl["Ly"], wl["params"], b=wl["b"], n_colours=wl["n_colours"],
              dt=wl["dt"], T=wl["T"], split=wl["split"], seed=wl.get("seed", 0), replica=replica)
    return s


def run_once(F, sim, wl):
    sim.init(1 if wl["init"] == "bernoulli" else 0, 0.5)
    sim.run_to_end()
    return sim.observe()


def cpu_baseline(wl, seconds):
    """Oracle events/s on a bounded sample: consecutive windows of replica 0
    from the workload's own initial state, until `seconds` of CPU time."""
    import numpy as np
    import oracle
    kind = wl["kind"]
    if kind == "flip":
        k_a, k_d, J, h, beta = wl["params"]
        model = oracle.Model("flip", wl["Lx"], wl["Ly"], k_a=k_a, k_d=k_d, J=J, h=h, beta=beta)
    else:
        y, k_r, D = wl["params"]
        model = oracle.Model("zgb", wl["Lx"], wl["Ly"], y=y, k_r=k_r, D=D)
    b = wl["b"]
    cmap = oracle.colour_map(model, b, b, wl["n_colours"])
    cols, durs, _ = oracle.schedule(wl["split"], wl["n_colours"], wl["dt"], wl["T"])
    if wl["init"] == "bernoulli":
        lat = oracle.init_bernoulli(model.N, 0.5, 0, 0)
    else:
        lat = np.zeros(model.N, np.uint8)
    t0 = time.process_time()
    w = 0
    events = 0
    chunk = 2
    while w < len(cols) and time.process_time() - t0 < seconds:
        n = min(chunk, len(cols) - w)
        res = oracle.fs_run(model, lat, b, b, cmap, wl["n_colours"], cols[w:w + n], durs[w:w + n], 0, 0, w0=w)
        lat = res["lattice"]
        events += res["events"]
        w += n
    el = time.process_time() - t0
    return {"value": events / el, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"{wl['name']}: windows [0,{w}) of {len(cols)} of replica 0, single-threaded, "
                      f"{events} events in {el:.1f} s CPU"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--J", type=float, default=1.0)
    ap.add_argument("--dt", type=float, default=0.1)
    ap.add_argument("--split", type=int, default=0)
    ap.add_argument("--timing-stride", type=int, default=8,
                    help="bracket every k-th sweep launch with HIP timing events")
    ap.add_argument("--waves-per-group", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    wl = workloads.c1(J=args.J, dt=args.dt, split=args.split)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = F.fskmc_ctx_create(0, stream.cuda_stream)
    F.fskmc_ctx_set_waves_per_group(ctx, args.waves_per_group)
    sims = [make_sim(F, ctx, wl, replica=i) for i in range(args.warmup + args.steps)]
    log(f"workload {wl['name']}: {sims[0].windows()[0]} windows per step")

    for i in range(args.warmup):
        run_once(F, sims[i], wl)
        log(f"warmup step {i} done")
    F.fskmc_sync(ctx)
    F.fskmc_ctx_read_kernel_timing(ctx)  # discard
    F.fskmc_ctx_set_kernel_timing(ctx, args.timing_stride)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obs = []
    for i in range(args.steps):
        obs.append(run_once(F, sims[args.warmup + i], wl))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_total, n_timed = F.fskmc_ctx_read_kernel_timing(ctx)
    F.fskmc_ctx_set_kernel_timing(ctx, 0)

    events = sum(o["events"] for o in obs)
    bw = sum(o["block_windows"] for o in obs)
    wr = sum(o["writes"] for o in obs)
    launches = sum(o["window"] for o in obs)
    log(f"timed {args.steps} steps: {el:.3f} s, {events} events, {launches} sweep launches, "
        f"{n_timed} timed launches avg {ms_total / max(n_timed, 1) * 1e3:.2f} us")
    bytes_per_launch = hbm_bytes(wl["kind"], wl["b"], bw, wr) / launches
    avg_launch_s = ms_total / 1e3 / max(n_timed, 1)
    achieved = bytes_per_launch / avg_launch_s / 1e9
    result = {
        "metric": METRIC,
        "value": events / el,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "lattice": [wl["Lx"], wl["Ly"]], "block": [wl["b"], wl["b"]],
                   "colours": wl["n_colours"], "windows_per_step": int(launches // args.steps),
                   "events_per_step": events / args.steps, "waves_per_group": args.waves_per_group},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_sweep_single<4,16,16,flip>", "bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": avg_launch_s * 1e6, "timed_launches": n_timed},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        result["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    for s in sims:
        s.close()
    F.fskmc_ctx_destroy(ctx)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
