"""Writes serial_refs.json: coverage and energy density of the exact serial
SSA (the oracle's part (a): the whole-lattice Markov chain of Sec. 1 eqs.
totalrate and skeleton) on the 1024^2 spin-flip lattice (Arrhenius rates,
h = 0, beta = 1, Bernoulli(1/2) start with key (7, r)) at J = 0.5, 1, 2,
sampled at t = 1, 2, 5, 10, 20, 50, 100, for replicas r = 0..31.  The GPU
splitting-error test compares the fractional-step scheme against these
replicas.

Run from the repository root:  python tests/golden/make_serial_refs.py [-j JOBS]
(each replica single-threaded; minutes per coupling)."""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle as orc  # noqa: E402

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "serial_refs.json")
L = 1024
SEED = 7
TIMES = (1.0, 2.0, 5.0, 10.0, 20.0, 50.0, 100.0)
REPLICAS = 32
COUPLINGS = (0.5, 1.0, 2.0)


def one(args):
    J, r = args
    m = orc.Model("flip", L, L, k_a=1.0, k_d=1.0, J=J, h=0.0, beta=1.0)
    lat0 = orc.init_bernoulli(L * L, 0.5, SEED, r)
    _, obs, ev = orc.ssa_serial(m, lat0, TIMES[-1] + 1e-9, SEED, r, list(TIMES))
    N = L * L
    return J, r, [float(v) / N for v in obs[:, 1]], [-J * float(v) / N for v in obs[:, 4]], int(ev)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=1)
    args = ap.parse_args()
    t0 = time.time()
    out = {"L": L, "seed": SEED, "times": list(TIMES), "replicas": REPLICAS, "model": "flip",
           "params": {"k_a": 1.0, "k_d": 1.0, "h": 0.0, "beta": 1.0}, "init": "bernoulli", "by_J": {}}
    work = [(J, r) for J in COUPLINGS for r in range(REPLICAS)]
    res = {}
    with ProcessPoolExecutor(max_workers=max(1, args.jobs)) as ex:
        for J, r, theta, energy, ev in ex.map(one, work):
            res[(J, r)] = (theta, energy, ev)
            print(f"J={J} r={r} events={ev} {time.time() - t0:.0f} s", flush=True)
    for J in COUPLINGS:
        out["by_J"][f"{J:g}"] = {"theta": [res[(J, r)][0] for r in range(REPLICAS)],
                                 "energy": [res[(J, r)][1] for r in range(REPLICAS)],
                                 "events": [res[(J, r)][2] for r in range(REPLICAS)]}
    with open(PATH, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")


if __name__ == "__main__":
    main()
