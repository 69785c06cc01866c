"""ctypes binding of libfskmc (include/fskmc.h).

The functions below carry the C names and only marshal arguments: every step
of the fractional-step path runs in the HIP library.  Importing this module
raises if libfskmc.so has not been built; there is no fallback.
"""
import atexit
import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FSKMC_LIB: another build of the same library (tests load a sanitized one)
LIB_PATH = os.environ.get("FSKMC_LIB") or os.path.join(_HERE, "libfskmc.so")

FSKMC_OK, FSKMC_EINVAL, FSKMC_ENOMEM, FSKMC_EDEVICE, FSKMC_EDECOMP, FSKMC_EBUSY, FSKMC_ESTATE = 0, -1, -2, -3, -4, -5, -6
FSKMC_MODEL_FLIP, FSKMC_MODEL_ZGB, FSKMC_MODEL_KAWASAKI = 1, 2, 3
MODELS = {"flip": FSKMC_MODEL_FLIP, "zgb": FSKMC_MODEL_ZGB, "kawasaki": FSKMC_MODEL_KAWASAKI}
FSKMC_LIE, FSKMC_STRANG, FSKMC_RANDOM = 0, 1, 2

ERRORS = {FSKMC_EINVAL: "EINVAL", FSKMC_ENOMEM: "ENOMEM", FSKMC_EDEVICE: "EDEVICE", FSKMC_EDECOMP: "EDECOMP",
          FSKMC_EBUSY: "EBUSY", FSKMC_ESTATE: "ESTATE"}


class FskmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class fskmc_lattice(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("Lx", ctypes.c_int), ("Ly", ctypes.c_int)]


class fskmc_flip_params(ctypes.Structure):
    _fields_ = [("k_a", ctypes.c_double), ("k_d", ctypes.c_double), ("J", ctypes.c_double),
                ("h", ctypes.c_double), ("beta", ctypes.c_double)]


class fskmc_zgb_params(ctypes.Structure):
    _fields_ = [("y", ctypes.c_double), ("k_r", ctypes.c_double), ("D", ctypes.c_double)]


class fskmc_kawasaki_params(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double), ("J", ctypes.c_double), ("beta", ctypes.c_double)]


class fskmc_nested(ctypes.Structure):
    _fields_ = [("bx", ctypes.c_int), ("by", ctypes.c_int), ("cx", ctypes.c_int), ("cy", ctypes.c_int),
                ("outer_colours", ctypes.c_int), ("inner_colours", ctypes.c_int), ("inner_split", ctypes.c_int),
                ("dtau", ctypes.c_double)]


class fskmc_decomp(ctypes.Structure):
    _fields_ = [("bx", ctypes.c_int), ("by", ctypes.c_int), ("n_colours", ctypes.c_int),
                ("colour_map", ctypes.POINTER(ctypes.c_int))]


class fskmc_schedule(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("T", ctypes.c_double), ("split", ctypes.c_int)]


class fskmc_key(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint32), ("replica", ctypes.c_uint32)]


class fskmc_obs(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int64), ("count", ctypes.c_int64 * 3), ("bonds_equal", ctypes.c_int64 * 3),
                ("bonds_ab", ctypes.c_int64), ("window", ctypes.c_uint64), ("steps", ctypes.c_uint64),
                ("events", ctypes.c_uint64), ("block_windows", ctypes.c_uint64), ("writes", ctypes.c_uint64),
                ("t", ctypes.c_double)]


SYMBOLS = [
    "fskmc_ctx_create", "fskmc_ctx_destroy", "fskmc_last_error", "fskmc_sim_create", "fskmc_sim_destroy",
    "fskmc_sim_attach_device_lattice", "fskmc_sim_init", "fskmc_sim_set_lattice", "fskmc_sim_get_lattice",
    "fskmc_sim_advance", "fskmc_sim_run_to_end", "fskmc_sim_windows", "fskmc_sim_observe",
    "fskmc_sim_block_events", "fskmc_sim_rate_table", "fskmc_sim_get_state", "fskmc_sim_set_state",
    "fskmc_sim_footprint", "fskmc_batch_advance", "fskmc_sync", "fskmc_ctx_set_waves_per_group",
    "fskmc_ctx_set_kernel_timing", "fskmc_ctx_read_kernel_timing", "fskmc_ctx_set_persistent",
    "fskmc_ctx_set_resident", "fskmc_ctx_set_wait_limit", "fskmc_ctx_set_rebalance", "fskmc_sim_workload",
    "fskmc_workload_partition", "fskmc_sim_last_partition", "fskmc_sim_create_nested", "fskmc_ctx_set_nested",
    "fskmc_ctx_set_batch_persistent", "fskmc_ctx_set_graphs", "fskmc_ctx_set_batch_streams",
    "fskmc_advance_noalloc",
]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libfskmc.so is not built ({LIB_PATH}); run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.fskmc_last_error.restype = ctypes.c_char_p
    L.fskmc_ctx_create.argtypes = [ctypes.c_int, vp, P(vp)]
    L.fskmc_ctx_destroy.argtypes = [vp]
    L.fskmc_ctx_set_waves_per_group.argtypes = [vp, ctypes.c_int]
    L.fskmc_sync.argtypes = [vp]
    L.fskmc_ctx_set_kernel_timing.argtypes = [vp, ctypes.c_int]
    L.fskmc_ctx_set_persistent.argtypes = [vp, ctypes.c_int]
    L.fskmc_ctx_set_resident.argtypes = [vp, ctypes.c_int]
    L.fskmc_ctx_set_wait_limit.argtypes = [vp, ctypes.c_double]
    L.fskmc_ctx_set_rebalance.argtypes = [vp, ctypes.c_int]
    L.fskmc_sim_workload.argtypes = [vp, P(ctypes.c_uint64), ctypes.c_size_t]
    L.fskmc_workload_partition.argtypes = [P(ctypes.c_uint64), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           P(ctypes.c_int32)]
    L.fskmc_sim_last_partition.argtypes = [vp, P(ctypes.c_int32), ctypes.c_size_t, P(ctypes.c_size_t)]
    L.fskmc_ctx_read_kernel_timing.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_uint64)]
    L.fskmc_sim_create.argtypes = [vp, P(fskmc_lattice), ctypes.c_int, vp, P(fskmc_decomp), P(fskmc_schedule),
                                   fskmc_key, P(vp)]
    L.fskmc_sim_create_nested.argtypes = [vp, P(fskmc_lattice), ctypes.c_int, vp, P(fskmc_nested),
                                          P(fskmc_schedule), fskmc_key, P(vp)]
    L.fskmc_ctx_set_nested.argtypes = [vp, ctypes.c_int]
    L.fskmc_ctx_set_batch_persistent.argtypes = [vp, ctypes.c_int]
    L.fskmc_ctx_set_graphs.argtypes = [vp, ctypes.c_int]
    L.fskmc_ctx_set_batch_streams.argtypes = [vp, ctypes.c_int]
    L.fskmc_sim_destroy.argtypes = [vp]
    L.fskmc_sim_attach_device_lattice.argtypes = [vp, vp, ctypes.c_size_t]
    L.fskmc_sim_init.argtypes = [vp, ctypes.c_int, ctypes.c_double]
    L.fskmc_sim_set_lattice.argtypes = [vp, P(ctypes.c_uint8), ctypes.c_size_t]
    L.fskmc_sim_get_lattice.argtypes = [vp, P(ctypes.c_uint8), ctypes.c_size_t]
    L.fskmc_sim_advance.argtypes = [vp, ctypes.c_uint64]
    L.fskmc_sim_run_to_end.argtypes = [vp]
    L.fskmc_sim_windows.argtypes = [vp, P(ctypes.c_uint64), P(ctypes.c_uint64)]
    L.fskmc_sim_observe.argtypes = [vp, P(fskmc_obs)]
    L.fskmc_sim_block_events.argtypes = [vp, P(ctypes.c_uint32), ctypes.c_size_t]
    L.fskmc_sim_rate_table.argtypes = [vp, P(ctypes.c_double), ctypes.c_size_t]
    L.fskmc_sim_get_state.argtypes = [vp, P(ctypes.c_uint64), P(ctypes.c_uint8), ctypes.c_size_t]
    L.fskmc_sim_set_state.argtypes = [vp, ctypes.c_uint64, P(ctypes.c_uint8), ctypes.c_size_t]
    L.fskmc_sim_footprint.argtypes = [P(fskmc_lattice), ctypes.c_int, P(fskmc_decomp), P(fskmc_schedule)]
    L.fskmc_sim_footprint.restype = ctypes.c_size_t
    L.fskmc_batch_advance.argtypes = [vp, P(vp), ctypes.c_int, ctypes.c_uint32]
    L.fskmc_advance_noalloc.argtypes = [ctypes.c_int, vp, P(fskmc_lattice), ctypes.c_int, vp, P(fskmc_decomp),
                                        P(fskmc_schedule), fskmc_key, vp, ctypes.c_uint64, ctypes.c_uint64, vp, vp]
    return L


lib = _load()


def _check(rc):
    if rc < 0:
        raise FskmcError(rc, lib.fskmc_last_error().decode())
    return rc


def _u8p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


# Contexts created through this module and the Sim objects made on each:
# fskmc_ctx_destroy releases a context's remaining simulations in the library,
# so their Python objects are closed here at the same moment (a later close()
# is then a no-op instead of a use of freed memory), and contexts still open
# when the interpreter exits are destroyed before the HIP runtime goes away.
_contexts = {}


def _ctx_key(ctx):
    return ctx.value if isinstance(ctx, ctypes.c_void_p) else int(ctx)


# --- thin wrappers with the C names -----------------------------------------
def fskmc_ctx_create(device=0, hip_stream=None):
    out = ctypes.c_void_p()
    _check(lib.fskmc_ctx_create(device, hip_stream, ctypes.byref(out)))
    _contexts[out.value] = weakref.WeakSet()
    return out


def fskmc_ctx_destroy(ctx):
    key = _ctx_key(ctx)
    for sim in list(_contexts.pop(key, ())):
        sim.handle = None  # released by the library together with the context
    _check(lib.fskmc_ctx_destroy(ctx))


@atexit.register
def _destroy_open_contexts():
    for key in list(_contexts):
        try:
            fskmc_ctx_destroy(ctypes.c_void_p(key))
        except Exception:
            pass


def fskmc_ctx_set_waves_per_group(ctx, waves):
    _check(lib.fskmc_ctx_set_waves_per_group(ctx, waves))


def fskmc_sync(ctx):
    _check(lib.fskmc_sync(ctx))


def fskmc_ctx_set_persistent(ctx, windows):
    _check(lib.fskmc_ctx_set_persistent(ctx, windows))


def fskmc_ctx_set_resident(ctx, on):
    _check(lib.fskmc_ctx_set_resident(ctx, 1 if on else 0))


def fskmc_ctx_set_wait_limit(ctx, seconds):
    _check(lib.fskmc_ctx_set_wait_limit(ctx, seconds))


def fskmc_ctx_set_rebalance(ctx, on):
    _check(lib.fskmc_ctx_set_rebalance(ctx, 1 if on else 0))


def fskmc_sim_workload(sim, n_blocks):
    a = np.empty(n_blocks, np.uint64)
    _check(lib.fskmc_sim_workload(sim, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n_blocks))
    return a


def fskmc_workload_partition(W, P, cap=0):
    W = np.ascontiguousarray(W, dtype=np.uint64)
    out = np.empty(P + 1, np.int32)
    _check(lib.fskmc_workload_partition(W.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), len(W), P, cap,
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return out


def fskmc_sim_last_partition(sim):
    n = ctypes.c_size_t()
    _check(lib.fskmc_sim_last_partition(sim, None, 0, ctypes.byref(n)))
    if n.value == 0:
        return None
    out = np.empty(n.value, np.int32)
    _check(lib.fskmc_sim_last_partition(sim, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n.value,
                                        ctypes.byref(n)))
    return out


def fskmc_ctx_set_kernel_timing(ctx, stride):
    _check(lib.fskmc_ctx_set_kernel_timing(ctx, stride))


def fskmc_ctx_read_kernel_timing(ctx):
    ms, n = ctypes.c_double(), ctypes.c_uint64()
    _check(lib.fskmc_ctx_read_kernel_timing(ctx, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def _decomp(bx, by, n_colours, colour_map):
    cm = None
    keep = None
    if colour_map is not None:
        keep = np.ascontiguousarray(colour_map, dtype=np.int32)
        cm = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    return fskmc_decomp(bx, by, n_colours, cm), keep


def _params(model, params):
    if model == FSKMC_MODEL_FLIP:
        return fskmc_flip_params(*params)
    if model == FSKMC_MODEL_KAWASAKI:
        return fskmc_kawasaki_params(*params)
    return fskmc_zgb_params(*params)


def fskmc_sim_create(ctx, dim, Lx, Ly, model, params, bx, by, n_colours, dt, T, split, seed, replica,
                     colour_map=None):
    lat = fskmc_lattice(dim, Lx, Ly)
    p = _params(model, params)
    dec, _keep = _decomp(bx, by, n_colours, colour_map)
    sch = fskmc_schedule(dt, T, split)
    out = ctypes.c_void_p()
    _check(lib.fskmc_sim_create(ctx, ctypes.byref(lat), model, ctypes.cast(ctypes.byref(p), ctypes.c_void_p),
                                ctypes.byref(dec), ctypes.byref(sch), fskmc_key(seed, replica), ctypes.byref(out)))
    return out


def fskmc_sim_create_nested(ctx, Lx, Ly, model, params, bx, by, cx, cy, outer_colours, inner_colours, inner_split,
                            dtau, dt, T, split, seed, replica):
    lat = fskmc_lattice(2, Lx, Ly)
    p = _params(model, params)
    nd = fskmc_nested(bx, by, cx, cy, outer_colours, inner_colours, inner_split, dtau)
    sch = fskmc_schedule(dt, T, split)
    out = ctypes.c_void_p()
    _check(lib.fskmc_sim_create_nested(ctx, ctypes.byref(lat), model, ctypes.cast(ctypes.byref(p), ctypes.c_void_p),
                                       ctypes.byref(nd), ctypes.byref(sch), fskmc_key(seed, replica),
                                       ctypes.byref(out)))
    return out


def fskmc_ctx_set_nested(ctx, on):
    _check(lib.fskmc_ctx_set_nested(ctx, 1 if on else 0))


def fskmc_ctx_set_batch_persistent(ctx, windows):
    _check(lib.fskmc_ctx_set_batch_persistent(ctx, int(windows)))


def fskmc_ctx_set_batch_streams(ctx, streams):
    _check(lib.fskmc_ctx_set_batch_streams(ctx, int(streams)))


def fskmc_ctx_set_graphs(ctx, on):
    _check(lib.fskmc_ctx_set_graphs(ctx, 1 if on else 0))


def fskmc_sim_destroy(sim):
    _check(lib.fskmc_sim_destroy(sim))


def fskmc_sim_attach_device_lattice(sim, dev_ptr, nbytes):
    _check(lib.fskmc_sim_attach_device_lattice(sim, ctypes.c_void_p(dev_ptr), nbytes))


def fskmc_sim_init(sim, kind, p=0.5):
    _check(lib.fskmc_sim_init(sim, kind, p))


def fskmc_sim_set_lattice(sim, host):
    a = np.ascontiguousarray(host, dtype=np.uint8).ravel()
    _check(lib.fskmc_sim_set_lattice(sim, _u8p(a), a.size))


def fskmc_sim_get_lattice(sim, n):
    a = np.empty(n, np.uint8)
    _check(lib.fskmc_sim_get_lattice(sim, _u8p(a), n))
    return a


def fskmc_sim_advance(sim, n_windows):
    _check(lib.fskmc_sim_advance(sim, n_windows))


def fskmc_sim_run_to_end(sim):
    _check(lib.fskmc_sim_run_to_end(sim))


def fskmc_sim_windows(sim):
    tot, nxt = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib.fskmc_sim_windows(sim, ctypes.byref(tot), ctypes.byref(nxt)))
    return tot.value, nxt.value


def fskmc_sim_observe(sim):
    o = fskmc_obs()
    _check(lib.fskmc_sim_observe(sim, ctypes.byref(o)))
    return {"n_sites": o.n_sites, "count": list(o.count), "bonds_equal": list(o.bonds_equal),
            "bonds_ab": o.bonds_ab, "window": o.window, "steps": o.steps, "events": o.events,
            "block_windows": o.block_windows, "writes": o.writes, "t": o.t}


def fskmc_sim_block_events(sim, n_blocks):
    a = np.empty(n_blocks, np.uint32)
    _check(lib.fskmc_sim_block_events(sim, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), n_blocks))
    return a


def fskmc_sim_rate_table(sim, cap=243 * 14):
    a = np.empty(cap, np.float64)
    n = _check(lib.fskmc_sim_rate_table(sim, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cap))
    return a[:n].copy()


def fskmc_sim_get_state(sim, n):
    a = np.empty(n, np.uint8)
    w = ctypes.c_uint64()
    _check(lib.fskmc_sim_get_state(sim, ctypes.byref(w), _u8p(a), n))
    return w.value, a


def fskmc_sim_set_state(sim, window, host):
    a = np.ascontiguousarray(host, dtype=np.uint8).ravel()
    _check(lib.fskmc_sim_set_state(sim, window, _u8p(a), a.size))


def fskmc_sim_footprint(dim, Lx, Ly, model, bx, by, n_colours, dt, T, split):
    lat = fskmc_lattice(dim, Lx, Ly)
    dec, _ = _decomp(bx, by, n_colours, None)
    sch = fskmc_schedule(dt, T, split)
    return lib.fskmc_sim_footprint(ctypes.byref(lat), model, ctypes.byref(dec), ctypes.byref(sch))


def fskmc_batch_advance(ctx, sims, windows):
    arr = (ctypes.c_void_p * len(sims))(*[s.value if isinstance(s, ctypes.c_void_p) else s for s in sims])
    _check(lib.fskmc_batch_advance(ctx, arr, len(sims), windows))


def fskmc_advance_noalloc(device, hip_stream, dim, Lx, Ly, model, params, bx, by, n_colours, dt, T, split, seed,
                          replica, d_lattice, w0, n_windows, d_block_events=None, d_events=None):
    """Device pointers (ints) for the lattice and the optional outputs."""
    lat = fskmc_lattice(dim, Lx, Ly)
    p = _params(model, params)
    dec, _ = _decomp(bx, by, n_colours, None)
    sch = fskmc_schedule(dt, T, split)
    _check(lib.fskmc_advance_noalloc(device, hip_stream, ctypes.byref(lat), model,
                                     ctypes.cast(ctypes.byref(p), ctypes.c_void_p), ctypes.byref(dec),
                                     ctypes.byref(sch), fskmc_key(seed, replica), ctypes.c_void_p(d_lattice), w0,
                                     n_windows, ctypes.c_void_p(d_block_events) if d_block_events else None,
                                     ctypes.c_void_p(d_events) if d_events else None))


# --- convenience object ------------------------------------------------------
class Sim:
    """One lattice simulation on the GPU.

    kind 'flip': params (k_a, k_d, J, h, beta); kind 'zgb': params (y, k_r, D);
    kind 'kawasaki': params (D, J, beta).  nested: a dict with keys cx, cy,
    outer_colours, inner_colours, inner_split and dtau for the nested
    decomposition (fskmc_sim_create_nested); n_colours is then ignored.
    """

    def __init__(self, ctx, kind, Lx, Ly=1, params=(1.0, 1.0, 0.0, 0.0, 1.0), b=None, bx=None, by=None,
                 n_colours=2, dt=0.1, T=1.0, split=FSKMC_LIE, seed=0, replica=0, colour_map=None, dim=None,
                 nested=None):
        self.ctx = ctx
        self.kind = kind
        self.dim = dim if dim is not None else (1 if Ly == 1 else 2)
        self.Lx, self.Ly = Lx, Ly
        if b is not None:
            bx, by = (b, b) if self.dim == 2 else (b, 1)
        self.bx, self.by = bx, by
        self.n_colours = n_colours
        if kind not in MODELS:
            raise ValueError(f"unknown model kind {kind!r}")
        self.model = MODELS[kind]
        if nested is not None:
            n = dict(nested)
            self.n_colours = n["outer_colours"] * n["inner_colours"]
            self.handle = fskmc_sim_create_nested(ctx, Lx, Ly, self.model, params, bx, by, n["cx"], n["cy"],
                                                  n["outer_colours"], n["inner_colours"], n["inner_split"],
                                                  n["dtau"], dt, T, split, seed, replica)
        else:
            self.handle = fskmc_sim_create(ctx, self.dim, Lx, Ly, self.model, params, bx, by, n_colours, dt, T,
                                           split, seed, replica, colour_map)
        self.N = Lx * Ly
        self.nb = (Lx // bx) * (Ly // by)
        live = _contexts.get(_ctx_key(ctx))
        if live is not None:
            live.add(self)

    def close(self):
        """Destroy the simulation; a no-op once closed or once its context
        has been destroyed (which released it)."""
        if self.handle is not None:
            handle, self.handle = self.handle, None
            fskmc_sim_destroy(handle)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, kind, p=0.5):
        fskmc_sim_init(self.handle, kind, p)

    def set_lattice(self, host):
        fskmc_sim_set_lattice(self.handle, host)

    def lattice(self):
        return fskmc_sim_get_lattice(self.handle, self.N)

    def advance(self, n):
        fskmc_sim_advance(self.handle, n)

    def run_to_end(self):
        fskmc_sim_run_to_end(self.handle)

    def windows(self):
        return fskmc_sim_windows(self.handle)

    def observe(self):
        return fskmc_sim_observe(self.handle)

    def workload(self):
        return fskmc_sim_workload(self.handle, self.nb)

    def last_partition(self):
        return fskmc_sim_last_partition(self.handle)

    def block_events(self):
        return fskmc_sim_block_events(self.handle, self.nb)

    def rate_table(self):
        return fskmc_sim_rate_table(self.handle)

    def get_state(self):
        return fskmc_sim_get_state(self.handle, self.N)

    def set_state(self, window, host):
        fskmc_sim_set_state(self.handle, window, host)
