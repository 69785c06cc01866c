"""Writes c3_jobs.json: the oracle's whole run (final-lattice SHA-256 and
accepted events; part (b), the blockwise scheme of Sec. 2.2 with the Lie
schedule of Sec. 2.2 eq. lie) of each of the 512 independent Ising replicas
of the batched workload (edges in {128, 256, 512, 1024}, J ~ U[0.2, 2],
h ~ U[-1, 1], beta = 1, Lie dt = 0.1, T = 10, Bernoulli(1/2) start, key (0, i))
with 16x16 blocks.  The benchmark compares its batched run of every job with
these values.

Run from the repository root:  python tests/golden/make_c3_jobs.py [-j JOBS]"""
import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as orc  # noqa: E402
from paper_1105_4673_amd import workloads  # noqa: E402  (seeded inputs only)

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_jobs.json")
B = 16


def one(job):
    k_a, k_d, J, h, beta = job["params"]
    m = orc.Model("flip", job["Lx"], job["Ly"], k_a=k_a, k_d=k_d, J=J, h=h, beta=beta)
    cmap = orc.colour_map(m, B, B, job["n_colours"])
    cols, durs, _ = orc.schedule(job["split"], job["n_colours"], job["dt"], job["T"], job["seed"], job["replica"])
    lat = orc.init_bernoulli(m.N, 0.5, job["seed"], job["replica"])
    res = orc.fs_run(m, lat, B, B, cmap, job["n_colours"], cols, durs, job["seed"], job["replica"])
    return f"{job['name']}_b{B}", {"sha256": hashlib.sha256(res["lattice"].tobytes()).hexdigest(),
                                   "events": int(res["events"]), "L": job["Lx"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=1)
    args = ap.parse_args()
    jobs = workloads.c3_jobs(n=512)
    # largest first, so the pool drains evenly
    jobs = sorted(jobs, key=lambda j: -j["Lx"] * j["Ly"])
    t0 = time.time()
    out = {}
    with ProcessPoolExecutor(max_workers=max(1, args.jobs)) as ex:
        for name, rec in ex.map(one, jobs):
            out[name] = rec
            if len(out) % 32 == 0:
                print(f"{len(out)} jobs, {time.time() - t0:.0f} s", flush=True)
    with open(PATH, "w") as f:
        json.dump({"block": B, "workload": "ising_x512_edges128-1024_b16_lie_dt0.1_T10", "jobs": out}, f, indent=0,
                  sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
