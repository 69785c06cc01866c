"""Oracle for the fractional-step lattice KMC method -- TEST INFRASTRUCTURE ONLY.

Plain, slow CPU reference implementations used to check the GPU library:

* ``fskmc_oracle.c`` (compiled with gcc into ``liboracle.so``):
  (a) the exact serial SSA of the whole-lattice Markov chain (Sec. 1, eqs.
  totalrate and skeleton; Sec. 2, eq. generator) and (b) the fractional-step
  scheme run block by block (Sec. 2.2, eqs. lie and exact; Sec. 3, eqs. strang,
  PCSl, PCSs, SLPCS) in the exact arithmetic that the GPU path reproduces.
* ``exact.py``: closed forms, finite transfer matrices and brute-force master
  equations that pin the oracle to the mathematics.
* ``balance.py``: the workload histogram's mass-transport map onto equal
  per-processor workloads (Sec. 6).

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with ``paper_1105_4673_amd``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fskmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# a planted-mistake variant built by tests/test_oracle_plants.py (test hook)
_LIB_OVERRIDE = os.environ.get("FSKMC_ORACLE_LIB")

MODEL_FLIP = 1
MODEL_ZGB = 2
MODEL_KAW = 3
LIE, STRANG, RANDOM = 0, 1, 2

GCC_FLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
             "-fexcess-precision=standard", "-Wall"]


def build(force=True, out=None, defines=(), extra_flags=()):
    """Compile the oracle's C part with gcc (test infrastructure).  `out`,
    `defines` and `extra_flags` build a variant (a planted mistake, a
    sanitized build) at another path."""
    if out is not None:
        subprocess.check_call(["gcc"] + GCC_FLAGS + list(extra_flags) + ["-D" + d for d in defines] +
                              ["-o", out, _SRC, "-lm"])
        return out
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc"] + GCC_FLAGS + ["-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class _Model(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("dim", ctypes.c_int), ("Lx", ctypes.c_int),
                ("Ly", ctypes.c_int), ("p", ctypes.c_double * 5)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        u32p, dblp, u8p, i64p, u64p, intp = (P(ctypes.c_uint32), P(ctypes.c_double), P(ctypes.c_uint8),
                                             P(ctypes.c_int64), P(ctypes.c_uint64), P(ctypes.c_int))
        L.or_philox.argtypes = [u32p, u32p, u32p]
        L.or_uniforms.argtypes = [u32p, dblp, dblp]
        L.or_log.argtypes = [ctypes.c_double]
        L.or_log.restype = ctypes.c_double
        L.or_site_rate.argtypes = [P(_Model), u8p, ctypes.c_int]
        L.or_site_rate.restype = ctypes.c_double
        L.or_rate_table.argtypes = [P(_Model), dblp, ctypes.c_int]
        L.or_tree_select.argtypes = [dblp, ctypes.c_int, ctypes.c_double, dblp, dblp]
        L.or_observe.argtypes = [P(_Model), u8p, i64p]
        L.or_init_bernoulli.argtypes = [u8p, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32]
        L.or_ssa_serial.argtypes = [P(_Model), u8p, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32,
                                    dblp, ctypes.c_int, i64p, u64p]
        L.or_decomp_check.argtypes = [P(_Model), ctypes.c_int, ctypes.c_int, ctypes.c_int, intp]
        L.or_schedule.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64, intp, dblp, u8p]
        L.or_schedule.restype = ctypes.c_int64
        L.or_fs_run.argtypes = [P(_Model), u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, intp,
                                intp, dblp, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                u32p, u8p, u8p, i64p, u64p]
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class Model:
    """A lattice model: 'flip' (Arrhenius adsorption/desorption, Sec. 7 eq.
    Arrhenius) with params (k_a, k_d, J, h, beta), 'zgb' (Sec. 7.1, Table
    COrates) with params (y, k_r, D), or 'kawasaki' (conserved spin exchange,
    Sec. 2 example, Arrhenius barrier of the moving particle) with params
    (D, J, beta)."""

    def __init__(self, kind, Lx, Ly=1, dim=None, **params):
        self.kind = kind
        self.Lx, self.Ly = int(Lx), int(Ly)
        self.dim = dim if dim is not None else (1 if Ly == 1 else 2)
        if kind == "flip":
            vals = [params.get("k_a", 1.0), params.get("k_d", 1.0), params.get("J", 0.0),
                    params.get("h", 0.0), params.get("beta", 1.0)]
            code = MODEL_FLIP
        elif kind == "zgb":
            vals = [params.get("y", 0.5), params.get("k_r", 1000.0), params.get("D", 0.0), 0.0, 0.0]
            code = MODEL_ZGB
        elif kind == "kawasaki":
            vals = [params.get("D", 1.0), params.get("J", 0.0), params.get("beta", 1.0), 0.0, 0.0]
            code = MODEL_KAW
        else:
            raise ValueError(kind)
        self.params = vals
        self._c = _Model(code, self.dim, self.Lx, self.Ly, (ctypes.c_double * 5)(*vals))

    @property
    def N(self):
        return self.Lx * self.Ly

    @property
    def z(self):
        return 2 if self.dim == 1 else 4

    @property
    def n_states(self):
        return 3 if self.kind == "zgb" else 2


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def uniforms(words):
    w = np.ascontiguousarray(words, dtype=np.uint32)
    U, V = ctypes.c_double(), ctypes.c_double()
    lib().or_uniforms(_ptr(w, ctypes.c_uint32), ctypes.byref(U), ctypes.byref(V))
    return U.value, V.value


def log(u):
    return lib().or_log(float(u))


def site_rate(model, lattice, site):
    lat = np.ascontiguousarray(lattice, dtype=np.uint8).ravel()
    return lib().or_site_rate(ctypes.byref(model._c), _ptr(lat, ctypes.c_uint8), int(site))


def rate_table(model):
    n = 2 * (model.z + 1) if model.kind == "flip" else 243 * 14
    out = np.zeros(n, np.float64)
    r = lib().or_rate_table(ctypes.byref(model._c), _ptr(out, ctypes.c_double), n)
    assert r == n, r
    return out


def tree_select(leaves, V):
    """(leaf index or -1, root, residual target) for the heap sum tree."""
    lv = np.ascontiguousarray(leaves, dtype=np.float64)
    root, resid = ctypes.c_double(), ctypes.c_double()
    i = lib().or_tree_select(_ptr(lv, ctypes.c_double), len(lv), float(V), ctypes.byref(root),
                             ctypes.byref(resid))
    return i, root.value, resid.value


def observe(model, lattice):
    lat = np.ascontiguousarray(lattice, dtype=np.uint8).ravel()
    out = np.zeros(7, np.int64)
    lib().or_observe(ctypes.byref(model._c), _ptr(lat, ctypes.c_uint8), _ptr(out, ctypes.c_int64))
    return out


def init_bernoulli(N, p, seed, replica):
    lat = np.zeros(N, np.uint8)
    lib().or_init_bernoulli(_ptr(lat, ctypes.c_uint8), int(N), float(p), seed, replica)
    return lat


def ssa_serial(model, lattice, T, seed, replica, sample_t):
    """Exact serial SSA.  Returns (final lattice, counts[n_samples, 7], events)."""
    lat = np.array(lattice, dtype=np.uint8).ravel().copy()
    st = np.ascontiguousarray(sample_t, dtype=np.float64)
    obs = np.zeros((len(st), 7), np.int64)
    ev = ctypes.c_uint64()
    r = lib().or_ssa_serial(ctypes.byref(model._c), _ptr(lat, ctypes.c_uint8), float(T), seed, replica,
                            _ptr(st, ctypes.c_double), len(st), _ptr(obs, ctypes.c_int64), ctypes.byref(ev))
    assert r == 0, r
    return lat, obs, ev.value


def decomp_check(model, bx, by, colour_map, n_colours):
    cm = np.ascontiguousarray(colour_map, dtype=np.int32).ravel()
    return lib().or_decomp_check(ctypes.byref(model._c), bx, by, n_colours, _ptr(cm, ctypes.c_int))


def colour_map(model, bx, by, n_colours):
    """Built-in colour maps: 2 colours (bi+bj)%2, 4 colours (bi%2)+2(bj%2)."""
    NBX, NBY = model.Lx // bx, model.Ly // by
    bi = np.arange(NBX)[None, :]
    bj = np.arange(NBY)[:, None]
    if n_colours == 2:
        cm = (bi + bj) % 2
    elif n_colours == 4:
        cm = (bi % 2) + 2 * (bj % 2)
    else:
        raise ValueError(n_colours)
    return np.ascontiguousarray(cm.ravel(), dtype=np.int32)


def schedule(split, n_colours, dt, T, seed=0, replica=0):
    """(colours[int32], durations[float64], step_end[uint8]) of all windows."""
    n = lib().or_schedule(split, n_colours, dt, T, seed, replica, 0, None, None, None)
    if n < 0:
        raise ValueError("invalid schedule (T/dt not an integer?)")
    cols = np.zeros(n, np.int32)
    durs = np.zeros(n, np.float64)
    ends = np.zeros(n, np.uint8)
    r = lib().or_schedule(split, n_colours, dt, T, seed, replica, n, _ptr(cols, ctypes.c_int),
                          _ptr(durs, ctypes.c_double), _ptr(ends, ctypes.c_uint8))
    assert r == n
    return cols, durs, ends


def fs_run(model, lattice, bx, by, cmap, n_colours, win_colour, win_dur, seed, replica, w0=0,
           want_W=False, want_snap=False, observe_flags=None):
    """Fractional-step scheme, block by block.  Returns a dict with the final
    lattice, total events and the optional per-window outputs."""
    lat = np.array(lattice, dtype=np.uint8).ravel().copy()
    cm = np.ascontiguousarray(cmap, dtype=np.int32)
    wc = np.ascontiguousarray(win_colour, dtype=np.int32)
    wd = np.ascontiguousarray(win_dur, dtype=np.float64)
    nw = len(wc)
    nb = (model.Lx // bx) * (model.Ly // by)
    W = np.zeros((nw, nb), np.uint32) if want_W else None
    snap = np.zeros((nw, model.N), np.uint8) if want_snap else None
    flags = None
    obs = None
    if observe_flags is not None:
        flags = np.ascontiguousarray(observe_flags, dtype=np.uint8)
        obs = np.zeros((int(flags.sum()), 7), np.int64)
    ev = ctypes.c_uint64()
    r = lib().or_fs_run(ctypes.byref(model._c), _ptr(lat, ctypes.c_uint8), bx, by, n_colours,
                        _ptr(cm, ctypes.c_int), _ptr(wc, ctypes.c_int), _ptr(wd, ctypes.c_double), nw, w0,
                        seed, replica,
                        _ptr(W, ctypes.c_uint32) if W is not None else None,
                        _ptr(snap, ctypes.c_uint8) if snap is not None else None,
                        _ptr(flags, ctypes.c_uint8) if flags is not None else None,
                        _ptr(obs, ctypes.c_int64) if obs is not None else None,
                        ctypes.byref(ev))
    assert r == 0, r
    return {"lattice": lat, "events": ev.value, "W": W, "snap": snap, "obs": obs}
