"""The oracle's result for a simulation job given as the GPU tests describe
it (kind, lattice, params, block edge, colours, dt, T, split, start, key):
the final lattice's SHA-256 and the accepted-event total of the blockwise
fractional-step scheme (Sec. 2.2 eq. exact, with the schedules of Sec. 3)
run to T.  Jobs too large for the oracle in seconds take their values from
tests/golden/full_runs.json, written by tests/golden/make_full_runs.py, which
calls only the oracle."""
import hashlib
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_cache = {}


def model_of(orc, kind, Lx, Ly, params):
    if kind == "flip":
        k_a, k_d, J, h, beta = params
        return orc.Model("flip", Lx, Ly, k_a=k_a, k_d=k_d, J=J, h=h, beta=beta)
    if kind == "kawasaki":
        D, J, beta = params
        return orc.Model("kawasaki", Lx, Ly, D=D, J=J, beta=beta)
    y, k_r, D = params
    return orc.Model("zgb", Lx, Ly, y=y, k_r=k_r, D=D)


def _key(spec):
    init = spec.get("init", "bernoulli")
    return (spec["kind"], spec["Lx"], spec["Ly"], tuple(float(p) for p in spec["params"]), spec["b"],
            spec["n_colours"], float(spec["dt"]), float(spec["T"]), int(spec["split"]), init,
            int(spec.get("seed", 0)), int(spec.get("replica", 0)))


def golden():
    with open(os.path.join(HERE, "golden", "full_runs.json")) as f:
        return json.load(f)


def _golden_lookup(spec):
    init = spec.get("init", "bernoulli")
    for g in golden().values():
        p = g["params"]
        prm = ((p["k_a"], p["k_d"], p["J"], p["h"], p["beta"]) if g["kind"] == "flip" else
               (p["D"], p["J"], p["beta"]) if g["kind"] == "kawasaki" else (p["y"], p["k_r"], p["D"]))
        Lx, Ly = g.get("Lx", g["L"]), g.get("Ly", g["L"])
        same = (g["kind"] == spec["kind"] and (Lx, Ly) == (spec["Lx"], spec["Ly"]) and
                tuple(map(float, prm)) == tuple(map(float, spec["params"])) and g["b"] == spec["b"] and
                g["n_colours"] == spec["n_colours"] and float(g["dt"]) == float(spec["dt"]) and
                float(g["T"]) == float(spec["T"]) and g["split"] == int(spec["split"]) and g["init"] == init and
                g["seed"] == int(spec.get("seed", 0)) and g["replica"] == int(spec.get("replica", 0)))
        if same and g.get("whole_run"):
            return g
    return None


def oracle_result(orc, spec, max_sites=1 << 18):
    """(sha256 of the final lattice, events) of the whole run of `spec`."""
    k = _key(spec)
    if k in _cache:
        return _cache[k]
    Lx, Ly = spec["Lx"], spec["Ly"]
    if Lx * Ly > max_sites:
        g = _golden_lookup(spec)
        if g is None:
            raise KeyError(f"no stored oracle value for a {Lx}x{Ly} job; add it to tests/golden/make_full_runs.py")
        out = (g["sha256"], g["events"])
    else:
        model = model_of(orc, spec["kind"], Lx, Ly, spec["params"])
        b = spec["b"]
        bx, by = (b, b) if Ly > 1 else (b, 1)
        seed, replica = int(spec.get("seed", 0)), int(spec.get("replica", 0))
        cmap = orc.colour_map(model, bx, by, spec["n_colours"])
        cols, durs, _ = orc.schedule(int(spec["split"]), spec["n_colours"], spec["dt"], spec["T"], seed, replica)
        if spec.get("init", "bernoulli") == "bernoulli":
            lat = orc.init_bernoulli(model.N, 0.5, seed, replica)
        else:
            lat = np.zeros(model.N, np.uint8)
        res = orc.fs_run(model, lat, bx, by, cmap, spec["n_colours"], cols, durs, seed, replica)
        out = (hashlib.sha256(res["lattice"].tobytes()).hexdigest(), int(res["events"]))
    _cache[k] = out
    return out
