/*
 * fskmc.h -- C ABI of libfskmc, a fractional-step parallel lattice kinetic
 * Monte Carlo library for AMD Instinct MI355X (gfx950).
 *
 * The method (Arampatzis, Katsoulakis, Plechac, Taufer, Xu, "Hierarchical
 * fractional-step approximations and parallel kinetic Monte Carlo
 * algorithms"): the generator of a lattice Markov jump process (Sec. 2,
 * eq. generator) is split over a colouring of the lattice into blocks
 * (Sec. 2.1, eqs. decomposition, sublatt, opdecomp).  A Trotter product
 * (Sec. 2.2, eq. lie; Sec. 3, eq. strang; Sec. 3.1, eq. SLPCS) turns the
 * evolution into a sequence of windows; in each window every block of the
 * active colour runs its own serial SSA kernel independently (eq. exact)
 * while all other sites are frozen (the three-stage step of Sec. 2.2).
 *
 * Conventions for every call:
 *  - Every function returns an int status: FSKMC_OK (0) or a negative code
 *    below.  The human-readable reason of the last failure on the calling
 *    thread is returned by fskmc_last_error().  Nothing throws across the ABI.
 *  - Handles are opaque; every create has a matching destroy.  Memory the
 *    library allocates it also frees.  Host buffers passed in are owned by the
 *    caller and copied before the call returns.
 *  - Sites are bytes, indexed y*Lx + x on a periodic Lx x Ly lattice (Ly = 1
 *    in 1D).  States: spin-flip {0,1}; reaction model {0 empty, 1 A, 2 B}.
 *  - Work is enqueued asynchronously on the context's HIP stream; calls that
 *    return host data synchronise that stream first.
 *  - Results are a pure function of (model, lattice, decomposition, schedule,
 *    key): the same inputs give the same bits whether a simulation is advanced
 *    alone or inside a batch.
 */
#ifndef FSKMC_H
#define FSKMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FSKMC_OK = 0,
    FSKMC_EINVAL = -1,  /* bad argument, shape or parameter                     */
    FSKMC_ENOMEM = -2,  /* host or device allocation failed / over budget       */
    FSKMC_EDEVICE = -3, /* a HIP runtime call failed                             */
    FSKMC_EDECOMP = -4, /* colour map does not tile or blocks of a colour interact */
    FSKMC_EBUSY = -5,   /* object still in use (e.g. a sim inside a running batch) */
    FSKMC_ESTATE = -6   /* call not valid in the current state (e.g. past T)     */
};

typedef struct fskmc_ctx fskmc_ctx; /* one GPU + one HIP stream            */
typedef struct fskmc_sim fskmc_sim; /* one lattice replica / job            */

/* Models (Sec. 2 examples; Sec. 7 eq. Arrhenius; Sec. 7.1 Table COrates). */
typedef enum {
    FSKMC_MODEL_FLIP = 1, /* Arrhenius adsorption/desorption spin flip, states {0,1} */
    FSKMC_MODEL_ZGB = 2,  /* A adsorption, B2 dissociative adsorption, A+B reaction,
                             A hopping; states {0,1=A,2=B}; pair events              */
    FSKMC_MODEL_KAWASAKI = 3 /* conserved spin exchange (Arrhenius surface diffusion),
                                states {0,1}; pair events; two-dimensional only      */
} fskmc_model;

/* Processor communication schedules (Sec. 3, eqs. PCSl, PCSs, SLPCS). */
typedef enum {
    FSKMC_LIE = 0,    /* per step: colours 0..K-1, each for dt                      */
    FSKMC_STRANG = 1, /* per step: 0..K-2 for dt/2, K-1 for dt, K-2..0 for dt/2     */
    FSKMC_RANDOM = 2  /* per step: K windows of dt, colour uniform from Philox (w,0,0,3) */
} fskmc_split;

/* Lattice Lambda_N (Sec. 2): dim 1 (Ly must be 1) or 2, periodic. */
typedef struct {
    int dim;
    int Lx, Ly;
} fskmc_lattice;

/* Spin-flip rates (Sec. 4.1 eq. adsdesrate with eq. potential; Sec. 7 eq.
 * Arrhenius): c(x) = k_a if sigma(x) = 0, and
 * k_d * exp(-(beta * (J * n + h))) if sigma(x) = 1, n = #occupied neighbours. */
typedef struct {
    double k_a, k_d, J, h, beta;
} fskmc_flip_params;

/* Reaction-model rates (Sec. 7.1, Table COrates), per site x and direction d:
 * A adsorption y; B2 dissociative adsorption on (x, x+e_d) (1-y)/4;
 * A+B -> 0+0 with x+e_d at k_r/4; A hop to an empty x+e_d at D/4. */
typedef struct {
    double y, k_r, D;
} fskmc_zgb_params;

/* Spin-exchange rates (Sec. 2, the conserved-dynamics example with the
 * Arrhenius barrier of Sec. 7 eq. Arrhenius): a particle at x moves to an
 * empty neighbour x+e_d at (D/4) * exp(-(beta * J * n)), n = #occupied
 * neighbours of x.  The particle number is invariant.  D >= 0; J, beta finite. */
typedef struct {
    double D, J, beta;
} fskmc_kawasaki_params;

/* Decomposition (Sec. 2.1): blocks of bx x by sites tile the lattice; block
 * m = bj*(Lx/bx) + bi.  colour_map (length #blocks, values in [0, n_colours))
 * may be NULL for the built-in maps: 2 colours (bi+bj)%2, 4 colours
 * (bi%2) + 2*(bj%2).  The GPU kernels need bx*by = 64*P with P in {1,4,16}
 * and either square blocks (8x8, 16x16, 32x32) or 1D rows (64P x 1). */
typedef struct {
    int bx, by, n_colours;
    const int* colour_map;
} fskmc_decomp;

/* Nested (hierarchical) decomposition (Sec. 5, eqs. sublatt2 and opdecomp2).
 * Coarse cells of cx x cy fine blocks (bx x by sites each) carry the outer
 * colouring over coarse positions (I, J): 2 colours (I+J)%2, 4 colours
 * (I%2)+2(J%2); inside a cell, fine blocks at (i, j) carry the inner colouring
 * (2 or 4 colours, the same formulas).  The scheme applies the schedule's
 * splitting (Lie or Strang, step dt) over the outer colours and replaces each
 * outer window of length d by the inner splitting (Lie or Strang, step dtau)
 * over the inner colours for time d; d / dtau must be an integer.  Fine block
 * m gets colour outer * inner_colours + inner, and window w of the expanded
 * list draws as in the flat scheme, so a nested sim gives the bits of a flat
 * sim with that colour map and window list. */
typedef struct {
    int bx, by;        /* fine blocks (one GPU wave each); the shapes of fskmc_decomp */
    int cx, cy;        /* fine blocks per coarse cell along x and y */
    int outer_colours; /* 2 or 4 */
    int inner_colours; /* 2 or 4 */
    int inner_split;   /* FSKMC_LIE or FSKMC_STRANG */
    double dtau;       /* inner step */
} fskmc_nested;

/* Schedule: window length dt and final time T (Sec. 2.2, T = n dt; T/dt must
 * be an integer to 1e-9 relative, and the run at most 2^31 - 2 windows, else
 * FSKMC_EINVAL). */
typedef struct {
    double dt, T;
    int split; /* fskmc_split */
} fskmc_schedule;

/* Philox4x32-10 key (Salmon et al., SC'11).  Draw e of block m in window w
 * uses counter (e, m, w, 0); the Bernoulli initial state uses (site, 0, 0, 1). */
typedef struct {
    uint32_t seed, replica;
} fskmc_key;

/* Integer observables at a window boundary (Sec. 7: coverage and two-point
 * correlations are derived from these counts on the host). */
typedef struct {
    int64_t n_sites;
    int64_t count[3];       /* sites per state                              */
    int64_t bonds_equal[3]; /* nearest-neighbour bonds (+x, +y) with both ends in state k */
    int64_t bonds_ab;       /* A-B bonds (reaction model)                    */
    uint64_t window;        /* windows completed                             */
    uint64_t steps;         /* complete fractional steps (t = steps * dt)    */
    uint64_t events;        /* accepted events since the last init/set_state */
    uint64_t block_windows; /* block-windows run since the last init/set_state */
    uint64_t writes;        /* block-windows with at least one event (written back) */
    double t;               /* physical time at the last complete step       */
} fskmc_obs;

/* Create a context on HIP device `device`.  hip_stream: an existing
 * hipStream_t (e.g. torch.cuda.current_stream().cuda_stream) used for all
 * work, or NULL for a library-owned stream.  out: receives the handle. */
int fskmc_ctx_create(int device, void* hip_stream, fskmc_ctx** out);
/* Wait for the context's stream, then destroy every simulation still created
 * on the context (their handles become invalid: do not pass them to
 * fskmc_sim_destroy afterwards) and the context itself.  A borrowed stream is
 * not destroyed. */
int fskmc_ctx_destroy(fskmc_ctx* ctx);

/* Message of the last failed call on this thread ("" if none).  The pointer
 * stays valid until the next failing call on the same thread. */
const char* fskmc_last_error(void);

/* Create one simulation: builds the FP64 rate table on the host, checks the
 * decomposition (FSKMC_EDECOMP if two blocks of one colour can interact:
 * spin flip writes C_m and reads C_m plus its neighbours; pair models read
 * and write C_m plus its neighbours), builds the window schedule and
 * allocates the device state.  params points at fskmc_flip_params,
 * fskmc_zgb_params or fskmc_kawasaki_params.  The lattice starts empty (all zeros).
 * The uploads go through a stream of the context's own (created on first use,
 * default priority): the call waits for them only, not for work already queued
 * on the context's stream. */
int fskmc_sim_create(fskmc_ctx* ctx, const fskmc_lattice* lattice, int model, const void* params,
                     const fskmc_decomp* decomp, const fskmc_schedule* schedule, fskmc_key key,
                     fskmc_sim** out);
int fskmc_sim_destroy(fskmc_sim* sim);

/* Create a simulation on a nested decomposition (see fskmc_nested); schedule
 * gives the outer step dt, T and the outer splitting (Lie or Strang).  Two
 * dimensions only.  FSKMC_EINVAL: cells that do not tile the block grid,
 * colourings other than 2 or 4, a random splitting, an outer window that is
 * not a whole number of inner steps.  FSKMC_EDECOMP: fewer than 2 x 2 coarse
 * cells, coarse cells of one outer colour that interact (pair models need 4
 * outer colours), or interacting fine blocks of one flat colour.  On a GPU,
 * square cells of 2 x 2 or 4 x 4 blocks (spin flip, 2 inner colours; or 4 x 4
 * blocks with 4; pair models 2 x 2 or 4 x 4 blocks with 4 inner colours) run
 * one launch per outer window, one workgroup per coarse cell, every inner
 * window inside it; for spin flip with fskmc_ctx_set_persistent(ctx, K > 0)
 * and the resident knob on, K windows run in one launch in which every cell
 * stays a resident workgroup and neighbouring cells exchange their one-site
 * boundary layers through tagged words between outer windows (when all
 * cells fit the device at once; waits are bounded as for the persistent
 * sweeps).  Other shapes, or fskmc_ctx_set_nested(ctx, 0), run the flat
 * sweeps on the same window list (same bits). */
int fskmc_sim_create_nested(fskmc_ctx* ctx, const fskmc_lattice* lattice, int model, const void* params,
                            const fskmc_nested* nested, const fskmc_schedule* schedule, fskmc_key key,
                            fskmc_sim** out);

/* Use caller-owned device memory (e.g. a torch uint8 tensor of Lx*Ly bytes)
 * as the lattice instead of the library's buffer.  The current lattice is
 * copied into it.  The buffer must outlive the sim. */
int fskmc_sim_attach_device_lattice(fskmc_sim* sim, void* dev_ptr, size_t bytes);

/* Initial state: kind 0 = empty, 1 = Bernoulli(p) per site from Philox
 * counter (site, 0, 0, 1).  Resets the window index and event counters. */
int fskmc_sim_init(fskmc_sim* sim, int kind, double p);

/* Copy a host lattice of n = Lx*Ly bytes in / out (get synchronises). */
int fskmc_sim_set_lattice(fskmc_sim* sim, const uint8_t* host, size_t n);
int fskmc_sim_get_lattice(fskmc_sim* sim, uint8_t* host, size_t n);

/* Enqueue the next n_windows windows of the schedule: one kernel launch per
 * window by default, up to K windows per persistent launch with
 * fskmc_ctx_set_persistent(ctx, K > 0), one launch per outer window for
 * nested sims.  FSKMC_ESTATE if that would pass the final time T, or if a
 * persistent launch of this sim aborted (see fskmc_ctx_set_wait_limit). */
int fskmc_sim_advance(fskmc_sim* sim, uint64_t n_windows);
/* Enqueue all remaining windows. */
int fskmc_sim_run_to_end(fskmc_sim* sim);
/* Number of windows in the schedule and the index of the next one. */
int fskmc_sim_windows(const fskmc_sim* sim, uint64_t* total, uint64_t* next);

/* Integer observables of the current lattice (synchronises). */
int fskmc_sim_observe(fskmc_sim* sim, fskmc_obs* out);

/* Accepted events per block in the last window each block ran (the workload
 * W of Sec. 6, eq. wload); n_blocks = (Lx/bx)*(Ly/by).  Synchronises. */
int fskmc_sim_block_events(fskmc_sim* sim, uint32_t* out, size_t n_blocks);

/* The host-built FP64 rate table.  Spin flip: 2*(z+1) entries [s*(z+1)+n];
 * reaction model: 243*14 entries [pattern*14 + c], 13 channels then the site
 * total, pattern = s + 3 nE + 9 nW + 27 nN + 81 nS.  n = capacity. */
int fskmc_sim_rate_table(const fskmc_sim* sim, double* out, size_t n);

/* Checkpoint / resume: the state is (lattice, next window index) because the
 * generator is counter-based.  get synchronises. */
int fskmc_sim_get_state(fskmc_sim* sim, uint64_t* window, uint8_t* host, size_t n);
int fskmc_sim_set_state(fskmc_sim* sim, uint64_t window, const uint8_t* host, size_t n);

/* Device bytes one simulation of this shape needs (admission control). */
size_t fskmc_sim_footprint(const fskmc_lattice* lattice, int model, const fskmc_decomp* decomp,
                           const fskmc_schedule* schedule);

/* Advance n simulations (same context) by up to `windows` windows each.
 * By default one launch per window: every launch runs the current window of
 * every sim that still has windows left, all blocks of all sims packed into
 * one grid.  With fskmc_ctx_set_batch_persistent(ctx, K > 0), K windows of
 * every sim run in one persistent launch whose waves take (window, job,
 * block) work items from a device counter in window order, each block
 * waiting only for the blocks it interacts with (Sec. 2.2 stage 2).  Sims
 * are grouped by kernel variant (model family, block shape); each group is
 * launched on its own, and with one packed launch per window launched
 * directly (graphs off) the groups run side by side on streams of their own
 * (fskmc_ctx_set_batch_streams), joined back into the context's stream before
 * the call's later work.  The launch sequence is captured as a HIP graph and
 * replayed by later calls with the same layout (fskmc_ctx_set_graphs).
 * Each sim's result is bit-identical to advancing it alone.  FSKMC_EDEVICE
 * at the next synchronising call if a persistent wait timed out (the lattices
 * of that batch are then unspecified). */
int fskmc_batch_advance(fskmc_ctx* ctx, fskmc_sim* const* sims, int n, uint32_t windows);

/* Knob that never changes results (default 0): windows per persistent
 * launch of fskmc_batch_advance; 0 = one packed launch per window. */
int fskmc_ctx_set_batch_persistent(fskmc_ctx* ctx, int windows);

/* Knob that never changes results (default 4): streams that the kernel-variant
 * groups of fskmc_batch_advance's packed launches are spread over (group i on
 * stream i mod streams; stream 0 is the context's, the others are created by
 * the library on first use, at the default priority, and destroyed with the
 * context).  Groups advance different sims, so their launches may overlap;
 * each group's windows stay in order on its stream.  1 = every launch on the
 * context's stream.  Persistent batched launches (fskmc_ctx_set_batch_persistent
 * > 0), launches replayed from a captured graph (fskmc_ctx_set_graphs on) and
 * launches sampled by kernel timing always use the context's stream.
 * FSKMC_EINVAL unless 1 <= streams <= 4. */
int fskmc_ctx_set_batch_streams(fskmc_ctx* ctx, int streams);

/* Knob that never changes results (default on): fskmc_batch_advance records
 * its launch sequence as a HIP graph once and replays it while the layout
 * stays the same (the same sims in the same order, window count per call and
 * knobs); the per-call job table is uploaded before each replay.  Off, and
 * while kernel timing is on, the launches go to the stream directly.  The
 * graph holds kernels only (counters and flags are cleared by kernels). */
int fskmc_ctx_set_graphs(fskmc_ctx* ctx, int on);

/* Wait for all work enqueued on the context's stream. */
int fskmc_sync(fskmc_ctx* ctx);

/* Knobs that never change results: waves (blocks) per workgroup for the sweep
 * kernels (1, 2, 4 or 8). */
int fskmc_ctx_set_waves_per_group(fskmc_ctx* ctx, int waves);

/* Knob that never changes results: with windows > 0, fskmc_sim_advance runs
 * up to `windows` windows of one simulation inside a single persistent
 * (cooperative) kernel in which each block waits only for the blocks it can
 * interact with (the local synchronisation of Sec. 2.2) instead of a kernel
 * boundary per window; 0 restores one launch per window.  A neighbour wait
 * longer than two seconds aborts the kernel and the next synchronising call
 * returns FSKMC_EDEVICE. */
int fskmc_ctx_set_persistent(fskmc_ctx* ctx, int windows);

/* Knob that never changes results (default on): persistent sweeps of spin-flip
 * simulations keep every block in LDS for the whole launch and exchange only
 * the blocks' one-site boundary layers between windows (Sec. 2.2, local
 * synchronisation), when the blocks fit the waves resident on the device (at
 * most eight blocks of 8x8 or 16x16 sites, or four of 32x32, per wave);
 * otherwise, and for the pair-event models, the
 * persistent sweep streams each block from HBM every window.  After a
 * persistent sweep returns FSKMC_EDEVICE the lattice contents are unspecified. */
int fskmc_ctx_set_resident(fskmc_ctx* ctx, int on);

/* Knob that never changes results (default off): resident persistent sweeps
 * give each wave a contiguous range of blocks (block order m = bj*NBX + bi)
 * by the mass-transport map (fskmc_workload_partition, capacity = the blocks
 * a wave holds: 8 for 8x8 and 16x16 blocks, 4 for 32x32) of the block costs
 * since the simulation's previous rebalanced launch, instead of fixed pairs.
 * A block's cost is its jumps in those windows plus 3 per window of its
 * colour there (a block-window's fixed work is about that of three jumps);
 * the first launch splits evenly.  The map is computed on the device between
 * launches, over max(ceil(n_blocks/2), ceil(n_blocks/capacity)) waves (at most
 * the resident waves). */
int fskmc_ctx_set_rebalance(fskmc_ctx* ctx, int on);

/* Knob that never changes results (default on): nested simulations whose
 * cells have a GPU variant advance one launch per outer window (one workgroup
 * per coarse cell, the inner windows separated by workgroup barriers); off,
 * they use the flat sweeps (one launch per window, or the persistent sweeps)
 * on the same window list.  With the persistent setting, spin-flip nested
 * sims use resident launches (see fskmc_sim_create_nested). */
int fskmc_ctx_set_nested(fskmc_ctx* ctx, int on);

/* Workload histogram (Sec. 6, eq. wload): out[m] = accepted events of block m
 * (block order m = bj*NBX + bi) since the last fskmc_sim_init, set_lattice or
 * set_state.  n_blocks must equal the simulation's block count.  Synchronises
 * the context's stream. */
int fskmc_sim_workload(fskmc_sim* sim, uint64_t* out, size_t n_blocks);

/* Mass-transport map of a workload histogram W[0..M) onto P processors
 * (Sec. 6, eq. wload and the map of its CDF onto equal masses):
 * bounds[0..P] (P+1 entries, caller-owned) with processor l owning blocks
 * [bounds[l], bounds[l+1]); bounds[l] is the first k with
 * P*(W[0] + ... + W[k-1]) >= l * total (a histogram without mass counts every
 * block once).  With cap > 0 every boundary is then clamped, in order l =
 * 1..P-1, into [max(bounds[l-1], M - (P-l)*cap), min(bounds[l-1] + cap, M)],
 * so no range holds more than cap blocks and the ranges still tile [0, M).
 * Host only.  FSKMC_EINVAL for M < 0, P < 1, cap < 0, NULL arrays or
 * M > P*cap. */
int fskmc_workload_partition(const uint64_t* W, int M, int P, int cap, int32_t* bounds);

/* The block ranges of the simulation's last rebalanced resident launch:
 * *n_out = number of boundaries (resident waves + 1; 0 if none yet), copied
 * to out when n >= *n_out; n = 0 only queries the size, 0 < n < *n_out is
 * FSKMC_EINVAL. */
int fskmc_sim_last_partition(const fskmc_sim* sim, int32_t* out, size_t n, size_t* n_out);

/* Failure handling: the longest time (seconds, in (0, 60], default 2) a block
 * of a persistent sweep waits for a neighbour before the sweep aborts; every
 * wave then leaves.  The context's abort flag is sticky: persistent launches
 * enqueued after the aborted one leave at their first wait, and the next
 * synchronising call (fskmc_sync, observe, get_lattice, get_state, workload,
 * block_events, last_partition) returns FSKMC_EDEVICE and clears the flag.
 * Every simulation a persistent launch advanced since the previous
 * synchronising call is then invalid: its lattice is unspecified and
 * advance, batch_advance, observe, get_lattice, get_state, workload and
 * block_events return FSKMC_ESTATE until fskmc_sim_init or
 * fskmc_sim_set_state.  Tiny values force the abort path (tests). */
int fskmc_ctx_set_wait_limit(fskmc_ctx* ctx, double seconds);

/* Measurement aid.  With stride > 0, every stride-th sweep launch on this
 * context is bracketed by two HIP timing events recorded on the context
 * stream (stride 0 turns it off).  read returns the summed duration of the
 * bracketed launches in milliseconds and their number since the previous
 * read, then forgets them; it synchronises the stream. */
int fskmc_ctx_set_kernel_timing(fskmc_ctx* ctx, int stride);
int fskmc_ctx_read_kernel_timing(fskmc_ctx* ctx, double* total_ms, uint64_t* n_launches);

/* Allocation-free advance, for callers that cannot allocate device memory at
 * call time: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It runs windows [w0, w0 + n_windows) of the scheme that
 * fskmc_sim_create would build from the same arguments, one launch per window
 * with the kernels of fskmc_sim_advance, on a lattice the caller owns, and
 * gives the same bits.
 *  - device, hip_stream: the GPU and a stream of that GPU the work is enqueued
 *    on (NULL = that device's null stream).  Asynchronous: nothing is waited for, and
 *    the only work enqueued is kernel launches (no allocation, copy or
 *    memset).  The calling thread's current device is switched to `device`
 *    for the call and restored before it returns; the first call on a device
 *    also looks up the array's device address (hipGetSymbolAddress).
 *  - lattice, model, params, schedule, key: as for fskmc_sim_create; decomp
 *    must use a built-in map (colour_map NULL, 2 or 4 colours).
 *  - d_lattice: device pointer, Lx*Ly bytes (site y*Lx + x), the state at
 *    window w0 on entry and after the last window on completion.
 *  - d_block_events: optional device pointer, n_blocks uint32 (block m =
 *    bj*NBX + bi): accepted events of each block's last window in this call,
 *    0 for blocks that ran none.  d_events: optional device pointer to one
 *    uint64, the call's accepted events.  Both written, not accumulated.
 * Working memory is a static device array of 1.36 MB per GPU (the rate
 * table, block lists and per-block counters), held until the process ends;
 * at most 65536 blocks per lattice (FSKMC_EINVAL beyond).  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.
 * FSKMC_EINVAL / FSKMC_EDECOMP as fskmc_sim_create, FSKMC_ESTATE if the
 * windows run past T, FSKMC_EDEVICE if a launch fails; arguments are checked
 * before any HIP call. */
int fskmc_advance_noalloc(int device, void* hip_stream, const fskmc_lattice* lattice, int model, const void* params,
                          const fskmc_decomp* decomp, const fskmc_schedule* schedule, fskmc_key key,
                          uint8_t* d_lattice, uint64_t w0, uint64_t n_windows, uint32_t* d_block_events,
                          unsigned long long* d_events);

#ifdef __cplusplus
}
#endif
#endif /* FSKMC_H */
