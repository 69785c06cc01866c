"""Seeded synthetic workloads (inputs only; no part of the method's arithmetic).

Shapes follow the paper's test problems: Ising-type spin-flip lattices with
Arrhenius rates (Sec. 7, eq. Arrhenius) and the A/B reaction lattice of
Sec. 7.1 (Table COrates).  The paper uses no dataset; every input here is a
lattice size, a parameter point and a Philox key.
"""
import numpy as np

# 64x64 spin flip, J=1, 8x8 blocks, 2 colours, Lie dt=0.1, T=10, empty start.
C0 = dict(name="ising64_b8_lie_dt0.1_T10", kind="flip", Lx=64, Ly=64, params=(1.0, 1.0, 1.0, 0.0, 1.0), b=8,
          n_colours=2, dt=0.1, T=10.0, split=0, init="empty")


def c1(J=1.0, dt=0.1, split=0, T=100.0):
    """1024^2 spin flip from Bernoulli(1/2), h=0, beta=1, 16x16 blocks."""
    sname = ["lie", "strang", "random"][split]
    return dict(name=f"ising1024_b16_J{J:g}_{sname}_dt{dt:g}_T{T:g}", kind="flip", Lx=1024, Ly=1024,
                params=(1.0, 1.0, J, 0.0, 1.0), b=16, n_colours=2, dt=dt, T=T, split=split, init="bernoulli")


def nested(c=2, dtau=0.05, T=20.0, dt=0.1, J=1.0):
    """The 1024^2 spin-flip lattice on a nested decomposition: coarse cells of
    c x c blocks of 16x16, 2 outer x 2 inner colours, outer Lie dt, inner Lie
    dtau, from Bernoulli(1/2)."""
    return dict(name=f"ising1024_b16_J{J:g}_nested_c{c}_lie{dt:g}_lie{dtau:g}_T{T:g}", kind="flip", Lx=1024,
                Ly=1024, params=(1.0, 1.0, J, 0.0, 1.0), b=16, dt=dt, T=T, split=0, init="bernoulli",
                nested=dict(cx=c, cy=c, outer_colours=2, inner_colours=2, inner_split=0, dtau=dtau))


def c2(y=0.5, D=10.0, T=10.0, L=4096):
    """4096^2 A/B reaction lattice, 32x32 blocks, 4 colours, Strang dt=0.05,
    empty start, k_r = 1e3."""
    return dict(name=f"reaction{L}_b32_y{y:g}_D{D:g}_strang_dt0.05_T{T:g}", kind="zgb", Lx=L, Ly=L,
                params=(y, 1000.0, D), b=32, n_colours=4, dt=0.05, T=T, split=1, init="empty")


def c3_jobs(n=512, seed=0, T=10.0, dt=0.1):
    """Independent Ising replicas: edge uniform in {128,256,512,1024},
    J ~ U[0.2, 2], h ~ U[-1, 1], beta = 1, Lie dt=0.1, key (0, i), 16x16 blocks."""
    rng = np.random.default_rng(seed)
    edges = rng.choice([128, 256, 512, 1024], size=n)
    J = rng.uniform(0.2, 2.0, size=n)
    h = rng.uniform(-1.0, 1.0, size=n)
    jobs = []
    for i in range(n):
        jobs.append(dict(name=f"c3job{i}", kind="flip", Lx=int(edges[i]), Ly=int(edges[i]),
                         params=(1.0, 1.0, float(J[i]), float(h[i]), 1.0), b=16, n_colours=2, dt=dt, T=T,
                         split=0, init="bernoulli", seed=0, replica=i))
    return jobs


def c4_requests(rate, n=256, seed=None, max_edge=2048):
    """Poisson request stream: arrival times at `rate` jobs/s; half Ising (Lie
    dt=0.1, 16x16 blocks), half A/B reaction (4-colour Strang dt=0.05, 16x16
    blocks); edge 64 * 32^u rounded to a multiple of 64 (log-uniform in
    [64, 2048]); T ~ U[10, 200] rounded to a multiple of dt.

    The block edge is the scheme's choice, not the model's.  Served jobs
    advance in lockstep, one window of every resident job per packed launch,
    so the last reaction jobs (up to 28000 windows) set the wall time with
    launches no longer than their slowest block's event chain; 16x16 blocks
    cut that chain to a quarter of the 32x32 blocks' sites."""
    rng = np.random.default_rng(int(rate) if seed is None else seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n):
        edge = int(round(64 * 32.0 ** rng.uniform(0, 1) / 64.0)) * 64
        edge = min(max(edge, 64), max_edge)
        T = float(rng.uniform(10, 200))
        if rng.uniform() < 0.5:
            dt = 0.1
            T = round(T / dt) * dt
            job = dict(kind="flip", Lx=edge, Ly=edge, params=(1.0, 1.0, float(rng.uniform(0.2, 2.0)),
                                                              float(rng.uniform(-1, 1)), 1.0),
                       b=16, n_colours=2, dt=dt, T=T, split=0, init="bernoulli")
        else:
            dt = 0.05
            T = round(T / dt) * dt
            job = dict(kind="zgb", Lx=edge, Ly=edge, params=(float(rng.choice([0.3, 0.5, 0.53])), 1000.0,
                                                             float(rng.choice([0.0, 10.0]))),
                       b=16, n_colours=4, dt=dt, T=T, split=1, init="empty")
        job.update(name=f"req{i}", arrival=float(arrivals[i]), seed=0, replica=i)
        reqs.append(job)
    return reqs


def half_filled(L=2048, J=1.0, dt=0.1, T=100.0):
    """L^2 spin flip, 16x16 blocks, Lie dt, the lower half of the rows empty
    and the upper half full: the empty half adsorbs at rate k_a while the full
    half hardly desorbs (k_d exp(-4 beta J)), a strongly unbalanced workload
    like the coverage gradient of the paper's rebalancing example."""
    return dict(name=f"ising{L}_b16_J{J:g}_lie_dt{dt:g}_half_filled", kind="flip", Lx=L, Ly=L,
                params=(1.0, 1.0, J, 0.0, 1.0), b=16, n_colours=2, dt=dt, T=T, split=0, init="half")
