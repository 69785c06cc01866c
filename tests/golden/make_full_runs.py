"""Writes full_runs.json: final-lattice SHA-256 and accepted-event totals of
fractional-step runs at the workloads' full sizes, computed by the oracle
alone (part (b), blockwise scheme of Sec. 2.2 with the schedules of Sec. 3).
The GPU tests and the benchmark's bit-exactness check compare the library's
runs against these values.

Run from the repository root:
    python tests/golden/make_full_runs.py [-j JOBS] [name ...]
(each case single-threaded, JOBS cases at a time; names given: recompute only
those cases; the JSON file is updated under a lock, so several invocations
may run at once)."""
import argparse
import fcntl
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor, as_completed

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as orc  # noqa: E402

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_runs.json")


def _flip(J, h=0.0):
    return dict(k_a=1.0, k_d=1.0, J=J, h=h, beta=1.0)


def _zgb(y, D):
    return dict(y=y, k_r=1000.0, D=D)


def _c1_cases():
    """The 1024^2 spin-flip grid (J in {0.5, 1, 2}, Lie and Strang, dt in
    {0.01, 0.1, 1}, T = 100, Bernoulli(1/2) start), replica 0 of each."""
    out = {}
    for J in (0.5, 1.0, 2.0):
        for split, sname in ((orc.LIE, "lie"), (orc.STRANG, "strang")):
            for dt in (0.01, 0.1, 1.0):
                name = f"ising1024_b16_J{J:g}_{sname}_dt{dt:g}_T100_r0"
                out[name] = ("flip", 1024, 1024, _flip(J), 16, 2, split, dt, 100.0, "bernoulli", 0, 0, None)
    return out


# name: kind, Lx, Ly, params, b, colours, split, dt, T, init, seed, replica, windows (None = whole run)
CASES = {
    "ising64_b8_J1_lie_dt0.1_T10_empty_r0": ("flip", 64, 64, _flip(1.0), 8, 2, orc.LIE, 0.1, 10.0, "empty", 0, 0,
                                             None),
    "ising1024_b16_J1_lie_dt0.1_T100_r0": ("flip", 1024, 1024, _flip(1.0), 16, 2, orc.LIE, 0.1, 100.0, "bernoulli",
                                           0, 0, None),
    "ising1024_b16_J0.5_strang_dt0.01_r7_w3000": ("flip", 1024, 1024, _flip(0.5), 16, 2, orc.STRANG, 0.01, 100.0,
                                                  "bernoulli", 0, 7, 3000),
    "ising1024_b16_J2_random_dt1_T100_r3": ("flip", 1024, 1024, _flip(2.0), 16, 2, orc.RANDOM, 1.0, 100.0,
                                            "bernoulli", 0, 3, None),
    "reaction4096_b32_y0.5_D10_strang_dt0.05_r1_w28": ("zgb", 4096, 4096, _zgb(0.5, 10.0), 32, 4, orc.STRANG, 0.05,
                                                       10.0, "empty", 0, 1, 28),
    "reaction4096_b32_y0.5_D10_strang_dt0.05_r1_w280": ("zgb", 4096, 4096, _zgb(0.5, 10.0), 32, 4, orc.STRANG,
                                                        0.05, 10.0, "empty", 0, 1, 280),
    # the timed 4096^2 reaction-lattice run (replica 0, whole run)
    "reaction4096_b32_y0.5_D10_strang_dt0.05_T10_r0": ("zgb", 4096, 4096, _zgb(0.5, 10.0), 32, 4, orc.STRANG, 0.05,
                                                       10.0, "empty", 0, 0, None),
    "reaction1024_b32_y0.5_D10_strang_dt0.05_T10_r1": ("zgb", 1024, 1024, _zgb(0.5, 10.0), 32, 4, orc.STRANG, 0.05,
                                                       10.0, "empty", 0, 1, None),
    # the 1024^2 job of the batched-kernel tests (whole run)
    "ising1024_b16_J1_lie_dt0.1_T1_r7": ("flip", 1024, 1024, _flip(1.0), 16, 2, orc.LIE, 0.1, 1.0, "bernoulli", 0, 7,
                                         None),
    # the full- and small-launch batched kernels' spin-flip job (whole run)
    "ising2112x2048_b32_J0.8_h-0.2_lie_dt0.2_T1_r21": ("flip", 2112, 2048, _flip(0.8, -0.2), 32, 2, orc.LIE, 0.2,
                                                       1.0, "bernoulli", 0, 21, None),
}
CASES.update(_c1_cases())


def run_case(kind, Lx, Ly, params, b, ncol, split, dt, T, init, seed, replica, windows):
    model = orc.Model(kind, Lx, Ly, **params)
    cmap = orc.colour_map(model, b, b, ncol)
    cols, durs, _ = orc.schedule(split, ncol, dt, T, seed, replica)
    whole = windows is None or windows >= len(cols)
    if windows is not None:
        cols, durs = cols[:windows], durs[:windows]
    if init == "bernoulli":
        lat = orc.init_bernoulli(model.N, 0.5, seed, replica)
    else:
        lat = np.zeros(model.N, np.uint8)
    res = orc.fs_run(model, lat, b, b, cmap, ncol, cols, durs, seed, replica)
    return {"kind": kind, "L": Lx, "Lx": Lx, "Ly": Ly, "params": params, "b": b, "n_colours": ncol, "split": split,
            "dt": dt, "T": T, "init": init, "seed": seed, "replica": replica, "windows": int(len(cols)),
            "whole_run": bool(whole), "events": int(res["events"]),
            "sha256": hashlib.sha256(res["lattice"].tobytes()).hexdigest()}


def _timed(name):
    t = time.time()
    return name, run_case(*CASES[name]), time.time() - t


def _store(name, rec):
    with open(PATH + ".lock", "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        out = {}
        if os.path.exists(PATH):
            with open(PATH) as f:
                out = json.load(f)
        out[name] = rec
        tmp = PATH + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
            f.write("\n")
        os.replace(tmp, PATH)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=1)
    ap.add_argument("names", nargs="*")
    args = ap.parse_args()
    names = args.names or list(CASES)
    for n in names:
        if n not in CASES:
            sys.exit(f"unknown case {n}")
    with ProcessPoolExecutor(max_workers=max(1, args.jobs)) as ex:
        futs = [ex.submit(_timed, n) for n in names]
        for f in as_completed(futs):
            name, rec, el = f.result()
            _store(name, rec)
            print(name, rec["events"], rec["sha256"][:16], f"{el:.1f} s", flush=True)


if __name__ == "__main__":
    main()
