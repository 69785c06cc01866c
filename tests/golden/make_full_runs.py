"""Writes full_runs.json: final-lattice SHA-256 and accepted-event totals of
whole fractional-step runs at the workloads' full sizes, computed by the
oracle alone (part (b), blockwise scheme of Sec. 2.2 with the schedules of
Sec. 3).  The GPU tests compare the library's runs against these values.

Run from the repository root:  python tests/golden/make_full_runs.py [name ...]
(single-threaded, several minutes; names given: recompute only those cases)."""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as orc  # noqa: E402

# name: kind, L, params, b, colours, split, dt, T, init, seed, replica, windows (None = whole run)
CASES = {
    "ising1024_b16_J1_lie_dt0.1_T100_r0": ("flip", 1024, dict(k_a=1.0, k_d=1.0, J=1.0, h=0.0, beta=1.0), 16, 2,
                                           orc.LIE, 0.1, 100.0, "bernoulli", 0, 0, None),
    "ising1024_b16_J0.5_strang_dt0.01_r7_w3000": ("flip", 1024, dict(k_a=1.0, k_d=1.0, J=0.5, h=0.0, beta=1.0),
                                                  16, 2, orc.STRANG, 0.01, 100.0, "bernoulli", 0, 7, 3000),
    "ising1024_b16_J2_random_dt1_T100_r3": ("flip", 1024, dict(k_a=1.0, k_d=1.0, J=2.0, h=0.0, beta=1.0), 16, 2,
                                            orc.RANDOM, 1.0, 100.0, "bernoulli", 0, 3, None),
    "reaction4096_b32_y0.5_D10_strang_dt0.05_r1_w28": ("zgb", 4096, dict(y=0.5, k_r=1000.0, D=10.0), 32, 4,
                                                       orc.STRANG, 0.05, 10.0, "empty", 0, 1, 28),
}


def run_case(kind, L, params, b, ncol, split, dt, T, init, seed, replica, windows):
    model = orc.Model(kind, L, L, **params)
    cmap = orc.colour_map(model, b, b, ncol)
    cols, durs, _ = orc.schedule(split, ncol, dt, T, seed, replica)
    if windows is not None:
        cols, durs = cols[:windows], durs[:windows]
    if init == "bernoulli":
        lat = orc.init_bernoulli(model.N, 0.5, seed, replica)
    else:
        lat = np.zeros(model.N, np.uint8)
    res = orc.fs_run(model, lat, b, b, cmap, ncol, cols, durs, seed, replica)
    return {"kind": kind, "L": L, "params": params, "b": b, "n_colours": ncol, "split": split, "dt": dt, "T": T,
            "init": init, "seed": seed, "replica": replica, "windows": int(len(cols)), "events": int(res["events"]),
            "sha256": hashlib.sha256(res["lattice"].tobytes()).hexdigest()}


def main():
    out = {}
    only = sys.argv[1:]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_runs.json")
    if only and os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    for name, case in CASES.items():
        if only and name not in only:
            continue
        t = time.time()
        out[name] = run_case(*case)
        print(name, out[name], f"{time.time() - t:.1f} s", flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
