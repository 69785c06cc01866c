// Host half of libfskmc: the C ABI declared in include/fskmc.h.
//
// Builds everything the kernels need before any launch -- the FP64 rate table
// (exp evaluated here, never on the device), the block decomposition with its
// independence check (Sec. 2.1), the window schedule (Sec. 2.2 eq. lie, Sec. 3
// eqs. strang, PCSl, PCSs, SLPCS) -- then drives one kernel launch per window.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fskmc.h"
#include "fskmc_decomp.h"
#include "fskmc_internal.h"
#include "fskmc_registry.h"

using namespace fskmc;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(FSKMC_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

// Philox4x32-10 on the host, for the random schedule's colour draws only.
void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = (uint32_t)p1;
        c[2] = n2;
        c[3] = (uint32_t)p0;
    }
}

}  // namespace

struct fskmc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int wpg = 2;
    unsigned long long* d_obs = nullptr;   // 9 counters
    unsigned long long* h_obs = nullptr;   // pinned
    // batched launches: packed job table and item -> job map (grown on demand)
    JobDesc* d_jobs = nullptr;
    size_t cap_jobs = 0;
    uint32_t* d_items = nullptr;
    size_t cap_items = 0;
    uint8_t* h_stage = nullptr;            // pinned staging for the uploads
    size_t cap_stage = 0;
    hipEvent_t stage_free = nullptr;
    // measurement aid: timing events around every timing_stride-th sweep launch
    int timing_stride = 0;
    uint64_t launch_counter = 0;
    std::vector<hipEvent_t> ev_pool; // pairs (start, stop)
    size_t ev_used = 0;              // pairs recorded since the last harvest
    double timed_ms = 0.0;
    uint64_t timed_n = 0;
    // persistent multi-window sweeps (0 = one launch per window)
    int persist = 0;
    bool resident = true;        // spin flip: keep blocks in LDS across the windows of a launch
    bool rebalance = false;      // resident launches: block ranges by the workload of the previous launch
    bool nested_kernel = true;   // nested sims: one workgroup per coarse cell and outer window
    unsigned long long wait_ticks = 200000000ull; // longest neighbour wait: 2 s of the 100 MHz wall clock
    // Raised by a persistent kernel on a timed-out wait and sticky: cleared
    // only by the synchronising call that reports it (check_abort).
    int32_t* d_abort = nullptr;
    int32_t* h_abort = nullptr;  // pinned copy, refreshed after each persistent launch
    SimRegistry<fskmc_sim> sims; // live sims, and those a pending persistent launch touched
    // batched advances: windows per persistent launch (0 = one packed launch
    // per window), HIP graph replay of the launch sequence, the work counter
    // of the persistent launches, and the cached graph with its layout key
    uint32_t batch_persist = 0;
    bool graphs = true;
    unsigned long long* d_queue = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<uint64_t> graph_key;
    // batched advances with several kernel-variant groups: streams on which
    // the groups' packed launches run side by side (created on first use),
    // forked from and joined back into `stream` by events
    int batch_streams = 4;
    // uploads of new simulations (created on first use): creating one waits
    // for its own uploads only, not for the work queued on `stream`
    hipStream_t upload = nullptr;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_join;
    hipEvent_t side_fork = nullptr;
};

struct fskmc_sim {
    fskmc_ctx* ctx = nullptr;
    // set when a persistent launch that advanced this sim aborted: the lattice
    // is unspecified until fskmc_sim_init or fskmc_sim_set_state
    bool invalid = false;
    int model = 0;
    fskmc_lattice lat{};
    double prm[5] = {0, 0, 0, 0, 0};
    int bx = 0, by = 0, n_colours = 0, NBX = 0, NBY = 0, nb = 0, P = 0, shape = 0;
    fskmc_schedule sched{};
    fskmc_key key{};
    std::vector<int> cmap;
    std::vector<int32_t> blocks;      // grouped by colour
    std::vector<int32_t> colour_off;  // n_colours + 1
    int max_per_colour = 0;
    std::vector<int8_t> win_colour;
    std::vector<double> win_dur;
    std::vector<uint8_t> step_end;
    uint64_t n_windows = 0, window = 0;
    uint64_t block_windows = 0; // since the last init / set_state
    std::vector<double> table;
    // device
    uint8_t* d_lat = nullptr;
    bool own_lat = true;
    double* d_table = nullptr;
    BlockCount* d_cnt = nullptr;
    int32_t* d_blocks = nullptr;
    int32_t* d_coff = nullptr;
    int8_t* d_wcol = nullptr;
    double* d_wdur = nullptr;
    // persistent sweep: colour per block, next window per colour, interacting
    // blocks, per-block epochs
    std::vector<int32_t> next_part;  // [n_colours][n_windows+1]
    int8_t* d_bcol = nullptr;
    int32_t* d_next = nullptr;
    int32_t* d_nbr = nullptr;
    int32_t* d_epoch = nullptr;
    // resident sweep: tagged edge words
    unsigned long long* d_edge = nullptr;
    // workload rebalancing: per-block events at the previous resident launch
    // and its windows, prefix-sum scratch, the block ranges of the last
    // rebalanced launch (n_owner boundaries)
    bool have_prev = false;
    uint64_t rb_w0 = 0;  // first window of the previous rebalanced launch
    unsigned long long* d_ev_prev = nullptr;
    unsigned long long* d_scan = nullptr;
    int32_t* d_owner = nullptr;
    size_t n_owner = 0, cap_owner = 0;
    // nested decomposition: coarse cells of cx x cy blocks (NCX per row),
    // k_outer x k_inner colours, inner scheme of step dtau; coarse cells
    // grouped by outer colour; per window, one past the last window of its
    // outer window
    bool nested = false, nest_kernel_ok = false;
    bool nest_resident_fits = true; // cleared when the cells cannot all be resident at once
    int cx = 0, cy = 0, NCX = 0, NCY = 0, k_outer = 0, k_inner = 0, inner_split = 0;
    double dtau = 0.0;
    std::vector<int32_t> cells, cell_off;
    std::vector<uint32_t> outer_end;
    std::vector<int32_t> ofirst, oidx;  // first window of each outer window (+ end); outer window of each window
    int32_t* d_cells = nullptr;
    int32_t* d_ofirst = nullptr;
};

namespace {

int64_t n_sites(const fskmc_lattice& L) { return (int64_t)L.Lx * L.Ly; }

int validate_lattice(const fskmc_lattice* L)
{
    if (!L)
        return fail(FSKMC_EINVAL, "lattice is NULL");
    if (L->dim != 1 && L->dim != 2)
        return fail(FSKMC_EINVAL, "dim must be 1 or 2 (got %d)", L->dim);
    if (L->Lx <= 0 || L->Ly <= 0)
        return fail(FSKMC_EINVAL, "lattice sizes must be positive");
    if (L->dim == 1 && L->Ly != 1)
        return fail(FSKMC_EINVAL, "a 1D lattice has Ly == 1");
    if ((int64_t)L->Lx * L->Ly > (int64_t)1 << 31)
        return fail(FSKMC_EINVAL, "lattice larger than 2^31 sites");
    return FSKMC_OK;
}

// GPU kernel variant for a block shape: P sites per lane, square or row.
int kernel_shape(const fskmc_lattice& L, int model, int bx, int by, int* P, int* shape)
{
    if (L.dim == 2) {
        if (bx != by || (bx != 8 && bx != 16 && bx != 32))
            return fail(FSKMC_EINVAL, "2D blocks must be 8x8, 16x16 or 32x32 (got %dx%d)", bx, by);
        *P = bx * by / 64;
        *shape = SHAPE_SQ;
    } else {
        if (model != FSKMC_MODEL_FLIP)
            return fail(FSKMC_EINVAL, "the pair-event models are two-dimensional");
        if (by != 1 || (bx != 64 && bx != 256 && bx != 1024))
            return fail(FSKMC_EINVAL, "1D blocks must be 64, 256 or 1024 sites (got %dx%d)", bx, by);
        *P = bx / 64;
        *shape = SHAPE_ROW;
    }
    return FSKMC_OK;
}

// Kernel family of a model: spin flip, or the table-driven pair-event sweep
// (the reaction model and spin exchange share it; only the table differs).
inline int kernel_model(int model)
{
    return model == FSKMC_MODEL_FLIP ? MODEL_FLIP : MODEL_ZGB;
}

// Independence of the blocks of each colour (Sec. 2.1, remark after eq.
// gendecomp), checked on the blocks' boundaries (fskmc_decomp.h).
int check_decomposition(const fskmc_sim& S)
{
    const DecompGeom G{S.lat.dim, S.lat.Lx, S.lat.Ly, S.bx, S.by, S.NBX};
    int c = -1;
    int64_t site = -1;
    if (decomp_conflict(G, S.model != FSKMC_MODEL_FLIP, S.n_colours, S.blocks.data(), S.colour_off.data(), &c, &site))
        return fail(FSKMC_EDECOMP, "blocks of colour %d interact at site %lld", c, (long long)site);
    return FSKMC_OK;
}

// Window i of a step of one splitting scheme over K colours with step dt; w is
// its index in the whole window list (the random schedule's Philox counter).
void scheme_window(int split, int K, double dt, fskmc_key key, int i, uint32_t w, int* c, double* d)
{
    if (split == FSKMC_LIE) {
        *c = i;
        *d = dt;
    } else if (split == FSKMC_STRANG) {
        *c = i < K ? i : 2 * (K - 1) - i;
        *d = *c == K - 1 ? dt : 0.5 * dt;
    } else {
        uint32_t ctr[4] = {w, 0u, 0u, 3u};
        philox_host(ctr, key.seed, key.replica);
        const uint64_t b = ((uint64_t)ctr[2] << 32) | ctr[3];
        const double V = (double)(b >> 11) * 0x1p-53;
        *c = (int)(V * (double)K);
        *d = dt;
    }
}

// Number of steps T / dt of a schedule (an integer within 1e-9, relative),
// and the windows per step of the splitting.
int scheme_steps(int split, int K, double dt, double T, int64_t* steps, int* per)
{
    if (!(dt > 0.0) || !(T >= 0.0) || !std::isfinite(dt) || !std::isfinite(T))
        return fail(FSKMC_EINVAL, "need dt > 0 and T >= 0");
    const double nd = std::floor(T / dt + 0.5);
    if (std::fabs(nd * dt - T) > 1e-9 * std::max(1.0, T))
        return fail(FSKMC_EINVAL, "T / dt = %.17g is not an integer", T / dt);
    if (split != FSKMC_LIE && split != FSKMC_STRANG && split != FSKMC_RANDOM)
        return fail(FSKMC_EINVAL, "unknown splitting %d", split);
    const int64_t max_windows = INT32_MAX - 1;
    *per = split == FSKMC_STRANG ? 2 * K - 1 : K;
    if (nd > (double)max_windows || (int64_t)nd * *per > max_windows)
        return fail(FSKMC_EINVAL, "more than %lld windows", (long long)max_windows);
    *steps = (int64_t)nd;
    return FSKMC_OK;
}

// Windows of one splitting scheme over K colours with step dt up to time T,
// appended to (col, dur, end); w0 is the index of the first of them in the
// whole list (the random schedule's Philox counter).
int scheme_windows(int split, int K, double dt, double T, fskmc_key key, uint64_t w0, std::vector<int8_t>& col,
                   std::vector<double>& dur, std::vector<uint8_t>& end)
{
    if (!(dt > 0.0) || !(T >= 0.0) || !std::isfinite(dt) || !std::isfinite(T))
        return fail(FSKMC_EINVAL, "need dt > 0 and T >= 0");
    const double nd = std::floor(T / dt + 0.5);
    if (std::fabs(nd * dt - T) > 1e-9 * std::max(1.0, T))
        return fail(FSKMC_EINVAL, "T / dt = %.17g is not an integer", T / dt);
    if (split != FSKMC_LIE && split != FSKMC_STRANG && split != FSKMC_RANDOM)
        return fail(FSKMC_EINVAL, "unknown splitting %d", split);
    // window indices, epochs and the per-colour next-window tables are 32-bit
    // signed on the device
    const int64_t max_windows = INT32_MAX - 1;
    const int per = split == FSKMC_STRANG ? 2 * K - 1 : K;
    if (nd > (double)max_windows || (int64_t)w0 + (int64_t)nd * per > max_windows)
        return fail(FSKMC_EINVAL, "more than %lld windows", (long long)max_windows);
    const int64_t steps = (int64_t)nd;
    col.reserve(col.size() + (size_t)(steps * per));
    dur.reserve(dur.size() + (size_t)(steps * per));
    uint32_t w = (uint32_t)w0;
    for (int64_t k = 0; k < steps; ++k) {
        for (int i = 0; i < per; ++i, ++w) {
            int c;
            double d;
            scheme_window(split, K, dt, key, i, w, &c, &d);
            col.push_back((int8_t)c);
            dur.push_back(d);
            end.push_back(i == per - 1 ? 1 : 0);
        }
    }
    return FSKMC_OK;
}

int build_schedule(fskmc_sim& S)
{
    S.win_colour.clear();
    S.win_dur.clear();
    S.step_end.clear();
    int rc = scheme_windows(S.sched.split, S.n_colours, S.sched.dt, S.sched.T, S.key, 0, S.win_colour, S.win_dur,
                            S.step_end);
    S.n_windows = S.win_colour.size();
    return rc;
}

// Nested scheme (Sec. 5, eqs. sublatt2 and opdecomp2): the outer scheme of
// step dt over the outer colours, each outer window (c, d) replaced by the
// inner scheme of step dtau over the inner colours for time d, on flat colour
// c * k_inner + inner colour.  step_end marks the end of every outer step.
int build_nested_schedule(fskmc_sim& S)
{
    if (S.sched.split == FSKMC_RANDOM || (S.inner_split != FSKMC_LIE && S.inner_split != FSKMC_STRANG))
        return fail(FSKMC_EINVAL, "the nested scheme takes Lie or Strang at both levels");
    std::vector<int8_t> oc;
    std::vector<double> od;
    std::vector<uint8_t> oe;
    int rc = scheme_windows(S.sched.split, S.k_outer, S.sched.dt, S.sched.T, S.key, 0, oc, od, oe);
    if (rc)
        return rc;
    S.win_colour.clear();
    S.win_dur.clear();
    S.step_end.clear();
    S.outer_end.clear();
    S.ofirst.clear();
    S.oidx.clear();
    for (size_t k = 0; k < oc.size(); ++k) {
        const size_t first = S.win_colour.size();
        if ((rc = scheme_windows(S.inner_split, S.k_inner, S.dtau, od[k], S.key, first, S.win_colour, S.win_dur,
                                 S.step_end)))
            return fail(rc, "outer window of length %.17g is not a whole number of inner steps %.17g (%s)", od[k],
                        S.dtau, fskmc_last_error());
        for (size_t i = first; i < S.win_colour.size(); ++i) {
            S.win_colour[i] = (int8_t)(oc[k] * S.k_inner + S.win_colour[i]);
            S.step_end[i] = 0;
        }
        S.step_end.back() = oe[k];
        S.outer_end.resize(S.win_colour.size(), (uint32_t)S.win_colour.size());
        S.ofirst.push_back((int32_t)first);
        S.oidx.resize(S.win_colour.size(), (int32_t)k);
    }
    S.ofirst.push_back((int32_t)S.win_colour.size());
    S.n_windows = S.win_colour.size();
    return FSKMC_OK;
}

// Entries of a model's rate table: 2 (z + 1) for spin flip, 243 x 14 for the
// pair-event models.
inline int table_size(int model, int dim)
{
    return model == FSKMC_MODEL_FLIP ? 2 * (2 * dim + 1) : 243 * 14;
}

// The FP64 rate table of a model into tab (table_size entries).
void fill_table(int model, int dim, const double prm[5], double* tab)
{
    std::fill(tab, tab + table_size(model, dim), 0.0);
    if (model == FSKMC_MODEL_FLIP) {
        const int z = dim == 1 ? 2 : 4;
        const double ka = prm[0], kd = prm[1], J = prm[2], h = prm[3], beta = prm[4];
        for (int n = 0; n <= z; ++n) {
            tab[n] = ka;
            tab[(z + 1) + n] = kd * std::exp(-(beta * (J * (double)n + h)));
        }
    } else if (model == FSKMC_MODEL_KAWASAKI) {
        // Exchange uses the hop channels 9..12 of the pair-event table; the
        // barrier counts the occupied neighbours of the moving particle.
        const double D = prm[0], J = prm[1], beta = prm[2];
        for (int pat = 0; pat < 243; ++pat) {
            int r = pat;
            const int s = r % 3;
            r /= 3;
            int nb[4], n = 0;
            for (int d = 0; d < 4; ++d) {
                nb[d] = r % 3;
                r /= 3;
                n += nb[d] == 1;
            }
            double* ch = &tab[(size_t)pat * 14];
            for (int d = 0; d < 4; ++d)
                if (s == 1 && nb[d] == 0)
                    ch[9 + d] = (D / 4.0) * std::exp(-(beta * (J * (double)n)));
            double tot = 0.0;
            for (int c = 0; c < 13; ++c)
                tot = tot + ch[c];
            ch[13] = tot;
        }
    } else {
        const double y = prm[0], kr = prm[1], D = prm[2];
        for (int pat = 0; pat < 243; ++pat) {
            int r = pat;
            const int s = r % 3;
            r /= 3;
            int nb[4];
            for (int d = 0; d < 4; ++d) { // E, W, N, S
                nb[d] = r % 3;
                r /= 3;
            }
            double* ch = &tab[(size_t)pat * 14];
            if (s == 0)
                ch[0] = y;
            for (int d = 0; d < 4; ++d) {
                if (s == 0 && nb[d] == 0)
                    ch[1 + d] = (1.0 - y) / 4.0;
                if ((s == 1 && nb[d] == 2) || (s == 2 && nb[d] == 1))
                    ch[5 + d] = kr / 4.0;
                if (s == 1 && nb[d] == 0)
                    ch[9 + d] = D / 4.0;
            }
            double tot = 0.0;
            for (int c = 0; c < 13; ++c)
                tot = tot + ch[c];
            ch[13] = tot;
        }
    }
}

void build_table(fskmc_sim& S)
{
    S.table.assign((size_t)table_size(S.model, S.lat.dim), 0.0);
    fill_table(S.model, S.lat.dim, S.prm, S.table.data());
}

// Every rate finite and small enough that a block's total stays finite (an
// infinite total would give zero waiting times and a window that never ends).
int check_table(const double* tab, int n)
{
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(tab[i]) || tab[i] < 0.0 || !std::isfinite(tab[i] * 4096.0))
            return fail(FSKMC_EINVAL, "rate %g is not finite or too large", tab[i]);
    return FSKMC_OK;
}

template <class T>
int dev_alloc(T** p, size_t count)
{
    *p = nullptr;
    if (count == 0)
        count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(FSKMC_ENOMEM, "hipMalloc(%zu bytes) failed: %s", count * sizeof(T), hipGetErrorString(e));
    }
    return FSKMC_OK;
}

void free_sim_device(fskmc_sim* S)
{
    if (S->own_lat && S->d_lat)
        (void)hipFree(S->d_lat);
    (void)hipFree(S->d_table);
    (void)hipFree(S->d_cnt);
    (void)hipFree(S->d_blocks);
    (void)hipFree(S->d_coff);
    (void)hipFree(S->d_wcol);
    (void)hipFree(S->d_wdur);
    (void)hipFree(S->d_bcol);
    (void)hipFree(S->d_next);
    (void)hipFree(S->d_nbr);
    (void)hipFree(S->d_epoch);
    (void)hipFree(S->d_edge);
    (void)hipFree(S->d_owner);
    (void)hipFree(S->d_cells);
    (void)hipFree(S->d_ofirst);
    (void)hipFree(S->d_ev_prev);
    (void)hipFree(S->d_scan);
    S->d_lat = nullptr;
}

// Sum the recorded timing pairs (synchronises the stream).
int harvest_timing(fskmc_ctx* c)
{
    if (c->ev_used == 0)
        return FSKMC_OK;
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < c->ev_used; ++i) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev_pool[2 * i], c->ev_pool[2 * i + 1]));
        c->timed_ms += ms;
        c->timed_n += 1;
    }
    c->ev_used = 0;
    return FSKMC_OK;
}

// Timing events for this launch (kernel-side start/stop), or none when the
// launch is not sampled.
LaunchTiming timing_begin(fskmc_ctx* c)
{
    LaunchTiming tm;
    if (c->timing_stride <= 0 || (c->launch_counter++ % (uint64_t)c->timing_stride) != 0)
        return tm;
    if (c->ev_used * 2 == c->ev_pool.size()) {
        if (c->ev_pool.size() >= 8192) {
            if (harvest_timing(c))
                return tm;
        } else {
            for (int k = 0; k < 256; ++k) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess)
                    return tm;
                c->ev_pool.push_back(e);
            }
        }
    }
    tm.start = c->ev_pool[2 * c->ev_used];
    tm.stop = c->ev_pool[2 * c->ev_used + 1];
    return tm;
}

void timing_end(fskmc_ctx* c, const LaunchTiming& tm)
{
    if (tm.start)
        c->ev_used++;
}

int reset_counters(fskmc_sim* S)
{
    hipStream_t st = S->ctx->stream;
    S->block_windows = 0;
    S->have_prev = false;
    HIP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(S->d_cnt), 2 * (int64_t)S->nb, 0ull, st));
    return FSKMC_OK;
}

// Inner windows [w0, w1) of one outer window of a nested sim: one launch,
// one workgroup per coarse cell of the outer colour.
int enqueue_nested(fskmc_sim* S, uint64_t w0, uint64_t w1)
{
    const int co = S->win_colour[w0] / S->k_inner;
    NestedArgs a{};
    a.lat = S->d_lat;
    a.table = S->d_table;
    a.cnt = S->d_cnt;
    a.win_colour = S->d_wcol;
    a.win_dur = S->d_wdur;
    a.cells = S->d_cells + S->cell_off[co];
    a.n_cells = S->cell_off[co + 1] - S->cell_off[co];
    a.Lx = S->lat.Lx;
    a.Ly = S->lat.Ly;
    a.NBX = S->NBX;
    a.NCX = S->NCX;
    a.k0 = S->key.seed;
    a.k1 = S->key.replica;
    a.w0 = (int)w0;
    a.w1 = (int)w1;
    const LaunchTiming tk = timing_begin(S->ctx);
    HIP_TRY(launch_sweep_nested(kernel_model(S->model), S->P, S->cx, S->k_inner, a, S->ctx->stream, tk));
    timing_end(S->ctx, tk);
    S->block_windows += (w1 - w0) * (uint64_t)a.n_cells * (uint64_t)(S->cx * S->cy / S->k_inner);
    return FSKMC_OK;
}

// Windows [w0, w1) of a nested spin-flip sim in one resident launch: 1 when
// the cells cannot all be resident at once (the caller launches per outer
// window instead).
int enqueue_nested_resident(fskmc_sim* S, uint64_t w0, uint64_t w1)
{
    fskmc_ctx* c = S->ctx;
    hipStream_t st = c->stream;
    const int cs = S->cx * S->bx;
    const int64_t words = (int64_t)S->NCX * S->NCY * (cs / 8);
    HIP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(S->d_edge), words, ~0ull, st));
    NestedResArgs a{};
    a.lat = S->d_lat;
    a.table = S->d_table;
    a.cnt = S->d_cnt;
    a.win_colour = S->d_wcol;
    a.win_dur = S->d_wdur;
    a.ofirst = S->d_ofirst;
    a.edge = S->d_edge;
    a.abort_flag = c->d_abort;
    a.Lx = S->lat.Lx;
    a.Ly = S->lat.Ly;
    a.NBX = S->NBX;
    a.NCX = S->NCX;
    a.NCY = S->NCY;
    a.k_outer = S->k_outer;
    a.k0 = S->key.seed;
    a.k1 = S->key.replica;
    a.w0 = (int)w0;
    a.w1 = (int)w1;
    a.ow0 = S->oidx[w0];
    a.ow1 = S->oidx[w1 - 1] + 1;
    a.wait_ticks = c->wait_ticks;
    const LaunchTiming tk = timing_begin(c);
    const hipError_t e = launch_sweep_nested_resident(S->P, S->cx, S->k_inner, a, st, tk);
    if (e == hipErrorInvalidConfiguration) {
        timing_end(c, LaunchTiming{});
        return 1;
    }
    HIP_TRY(e);
    timing_end(c, tk);
    HIP_TRY(hipMemcpyAsync(c->h_abort, c->d_abort, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    c->sims.touched(S);
    for (uint64_t w = w0; w < w1; ++w) {
        const int co = S->win_colour[w] / S->k_inner;
        S->block_windows += (uint64_t)(S->cell_off[co + 1] - S->cell_off[co]) * (uint64_t)(S->cx * S->cy / S->k_inner);
    }
    return FSKMC_OK;
}

int enqueue_window(fskmc_sim* S, uint64_t w)
{
    const int c = S->win_colour[w];
    SweepArgs a;
    a.lat = S->d_lat;
    a.table = S->d_table;
    a.cnt = S->d_cnt;
    a.blocks = S->d_blocks + S->colour_off[c];
    a.n_blocks = S->colour_off[c + 1] - S->colour_off[c];
    a.Lx = S->lat.Lx;
    a.Ly = S->lat.Ly;
    a.NBX = S->NBX;
    a.k0 = S->key.seed;
    a.k1 = S->key.replica;
    a.w = (uint32_t)w;
    a.dur = S->win_dur[w];
    const LaunchTiming tk = timing_begin(S->ctx);
    HIP_TRY(launch_sweep_single(kernel_model(S->model), S->P, S->shape, S->ctx->wpg, a, S->ctx->stream, tk));
    timing_end(S->ctx, tk);
    S->block_windows += (uint64_t)a.n_blocks;
    return FSKMC_OK;
}

// Windows [w0, w1) in one persistent kernel: epochs set to each block's first
// window >= w0, one cooperative launch, and the (sticky) abort flag copied
// back for the next synchronising call to check.
int enqueue_persistent(fskmc_sim* S, uint64_t w0, uint64_t w1)
{
    fskmc_ctx* c = S->ctx;
    hipStream_t st = c->stream;
    HIP_TRY(launch_epoch_init(S->d_epoch, S->d_bcol, S->d_next, S->nb, (int)S->n_windows, (int)w0, st));
    PersistArgs a;
    a.lat = S->d_lat;
    a.table = S->d_table;
    a.cnt = S->d_cnt;
    a.blocks = S->d_blocks;
    a.colour_off = S->d_coff;
    a.win_colour = S->d_wcol;
    a.win_dur = S->d_wdur;
    a.next_part = S->d_next;
    a.nbr = S->d_nbr;
    a.epoch = S->d_epoch;
    a.abort_flag = c->d_abort;
    a.Lx = S->lat.Lx;
    a.Ly = S->lat.Ly;
    a.NBX = S->NBX;
    a.k0 = S->key.seed;
    a.k1 = S->key.replica;
    a.n_windows = (int)S->n_windows;
    a.w0 = (int)w0;
    a.w1 = (int)w1;
    a.n_waves = 0;
    a.wait_ticks = c->wait_ticks;
    const LaunchTiming tk = timing_begin(c);
    HIP_TRY(launch_sweep_persistent(kernel_model(S->model), S->P, S->shape, c->wpg, a, S->max_per_colour, st, tk));
    timing_end(c, tk);
    HIP_TRY(hipMemcpyAsync(c->h_abort, c->d_abort, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    c->sims.touched(S);
    for (uint64_t w = w0; w < w1; ++w) {
        const int col = S->win_colour[w];
        S->block_windows += (uint64_t)(S->colour_off[col + 1] - S->colour_off[col]);
    }
    return FSKMC_OK;
}

// Mass-transport map of a workload histogram onto P processors (Sec. 6):
// boundary l is the first k with P * (W[0] + ... + W[k-1]) >= l * total (a
// histogram without mass counts every block once), clamped in order into
// [max(b_{l-1}, M - (P-l) cap), min(b_{l-1} + cap, M)] when a capacity is
// given.
void cdf_ranges(const uint64_t* W, int M, int P, int cap, int32_t* bounds)
{
    unsigned __int128 total = 0;
    for (int m = 0; m < M; ++m)
        total += W[m];
    const bool flat = total == 0;
    if (flat)
        total = (unsigned)M;
    bounds[0] = 0;
    unsigned __int128 cum = 0;
    int k = 0;
    for (int l = 1; l < P; ++l) {
        const unsigned __int128 target = (unsigned __int128)l * total;
        while (k < M && cum * (unsigned)P < target) {
            cum += flat ? 1u : W[k];
            ++k;
        }
        int64_t b = k;
        if (cap > 0) {
            const int64_t prev = bounds[l - 1];
            const int64_t lo = std::max<int64_t>(prev, (int64_t)M - (int64_t)(P - l) * cap);
            const int64_t hi = std::min<int64_t>(prev + cap, M);
            b = std::min(std::max(b, lo), hi);
        }
        bounds[l] = (int32_t)b;
    }
    bounds[P] = M;
}

// Fixed cost of one block-window in units of one jump's cost, the block cost
// of the rebalancing map (measured: staging, tree build and edge exchange
// take about as long as three events).
constexpr unsigned long long kWindowCost = 3;

// Block ranges of the next resident launch, computed on the device from the
// workload since the previous rebalanced launch (an even split the first
// time; otherwise the jumps of windows [previous start, w0) plus kWindowCost
// per window of the block's colour in that range) over as many waves as an
// even split would use (two blocks per wave, more if the lattice needs it),
// each range at most the wave's capacity; the remaining resident waves get
// empty ranges.  Returns 1 when the blocks do not fit the resident waves.
int rebalance_ranges(fskmc_sim* S, uint64_t w0)
{
    fskmc_ctx* c = S->ctx;
    const int waves = resident_waves(S->P, S->shape, c->wpg);
    const int cap = resident_capacity(S->P);
    if (waves <= 0 || (int64_t)S->nb > (int64_t)waves * cap)
        return 1;
    if (!S->d_ev_prev) {
        if (int rc = dev_alloc(&S->d_ev_prev, S->nb))
            return rc;
        if (int rc = dev_alloc(&S->d_scan, S->nb))
            return rc;
    }
    if (S->cap_owner < (size_t)waves + 1) {
        (void)hipFree(S->d_owner);
        S->d_owner = nullptr;
        S->cap_owner = 0;
        if (int rc = dev_alloc(&S->d_owner, (size_t)waves + 1))
            return rc;
        S->cap_owner = (size_t)waves + 1;
    }
    const int use = std::min(waves, std::max((S->nb + 1) / 2, (S->nb + cap - 1) / cap));
    // the jumps since the previous rebalanced launch cover windows [rb_w0, w0)
    HIP_TRY(launch_rebalance(S->d_cnt, S->d_ev_prev, S->d_bcol, S->d_wcol, (int)S->rb_w0, (int)w0,
                             S->have_prev ? 0 : 1, kWindowCost, S->d_scan, S->d_owner, S->nb, use, waves, cap,
                             c->stream));
    S->have_prev = true;
    S->rb_w0 = w0;
    S->n_owner = (size_t)waves + 1;
    return FSKMC_OK;
}

// Windows [w0, w1) of a spin-flip simulation in one resident launch: edge
// tags set to a value no window expects, one cooperative launch.  Returns 1 (nothing enqueued but the fill) when the
// blocks do not fit the resident waves; the caller then streams.
int enqueue_resident(fskmc_sim* S, uint64_t w0, uint64_t w1)
{
    fskmc_ctx* c = S->ctx;
    hipStream_t st = c->stream;
    HIP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(S->d_edge), 4 * (int64_t)S->nb, ~0ull, st));
    ResidentArgs a;
    a.lat = S->d_lat;
    a.table = S->d_table;
    a.cnt = S->d_cnt;
    a.bcol = S->d_bcol;
    a.win_colour = S->d_wcol;
    a.win_dur = S->d_wdur;
    a.edge = S->d_edge;
    a.abort_flag = c->d_abort;
    a.Lx = S->lat.Lx;
    a.Ly = S->lat.Ly;
    a.NBX = S->NBX;
    a.NBY = S->NBY;
    a.nb = S->nb;
    a.k0 = S->key.seed;
    a.k1 = S->key.replica;
    a.n_windows = (int)S->n_windows;
    a.w0 = (int)w0;
    a.w1 = (int)w1;
    a.n_waves = 0;
    a.bpw = 0;
    a.owner = nullptr;
    a.wait_ticks = c->wait_ticks;
    if (c->rebalance) {
        int rc = rebalance_ranges(S, w0);
        if (rc == 1)
            return 1;
        if (rc)
            return rc;
        a.owner = S->d_owner;
        a.n_waves = (int)S->n_owner - 1;
    }
    const LaunchTiming tk = timing_begin(c);
    const hipError_t e = launch_sweep_resident(S->P, S->shape, c->wpg, a, st, tk);
    if (e == hipErrorInvalidConfiguration) {
        timing_end(c, LaunchTiming{});
        return 1;
    }
    HIP_TRY(e);
    timing_end(c, tk);
    HIP_TRY(hipMemcpyAsync(c->h_abort, c->d_abort, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    c->sims.touched(S);
    for (uint64_t w = w0; w < w1; ++w) {
        const int col = S->win_colour[w];
        S->block_windows += (uint64_t)(S->colour_off[col + 1] - S->colour_off[col]);
    }
    return FSKMC_OK;
}

// After a stream synchronisation: did a persistent sweep abort since the
// last check?  The flag is sticky on the device, so the copy taken after the
// last persistent launch sees an abort of any earlier one.  On an abort every
// sim a persistent launch advanced since the last check is marked invalid,
// and the flag is cleared for the launches that follow.
int check_abort(fskmc_ctx* c)
{
    const bool aborted = c->h_abort && *c->h_abort;
    for (fskmc_sim* S : c->sims.settle(aborted))
        S->invalid = true;
    if (!aborted)
        return FSKMC_OK;
    *c->h_abort = 0;
    HIP_TRY(launch_fill_u32(reinterpret_cast<uint32_t*>(c->d_abort), 1, 0u, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return fail(FSKMC_EDEVICE, "persistent sweep aborted: a neighbour wait timed out");
}

int check_valid(const fskmc_sim* S)
{
    if (S->invalid)
        return fail(FSKMC_ESTATE, "a persistent sweep of this simulation aborted: its lattice is unspecified until "
                                  "fskmc_sim_init or fskmc_sim_set_state");
    return FSKMC_OK;
}

// Blocks that can interact with block m (their read/write sets meet): the
// four edge neighbours for spin flip (the two in 1D), the eight surrounding
// blocks for pair events.  Self and repeats (small periodic grids) dropped.
void build_neighbours(const fskmc_sim& S, std::vector<int32_t>& nbr)
{
    nbr.assign((size_t)S.nb * 8, -1);
    const bool pair = S.model != FSKMC_MODEL_FLIP;
    for (int m = 0; m < S.nb; ++m) {
        const int bi = m % S.NBX, bj = m / S.NBX;
        int k = 0;
        for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di) {
                if (di == 0 && dj == 0)
                    continue;
                if (!pair && di != 0 && dj != 0)
                    continue;
                if (S.NBY == 1 && dj != 0)
                    continue;
                const int ni = (bi + di + S.NBX) % S.NBX, nj = (bj + dj + S.NBY) % S.NBY;
                const int n = nj * S.NBX + ni;
                if (n == m)
                    continue;
                bool seen = false;
                for (int q = 0; q < k; ++q)
                    seen = seen || nbr[(size_t)m * 8 + q] == n;
                if (!seen)
                    nbr[(size_t)m * 8 + k++] = n;
            }
    }
}

size_t footprint_of(int64_t N, int model, int nb, uint64_t n_windows, int n_colours)
{
    const size_t tab = model == FSKMC_MODEL_FLIP ? 10 * 8 : 243 * 14 * 8;
    return (size_t)N + tab + (size_t)nb * (sizeof(BlockCount) + 4 + 1 + 32 + 4) + (size_t)(n_colours + 1) * 4 +
           (size_t)n_windows * (1 + 8) + (size_t)n_colours * (n_windows + 1) * 4;
}

}  // namespace

extern "C" {

const char* fskmc_last_error(void) { return g_err.c_str(); }

int fskmc_ctx_create(int device, void* hip_stream, fskmc_ctx** out)
{
    if (!out)
        return fail(FSKMC_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return fail(FSKMC_EINVAL, "device %d out of range (%d devices)", device, ndev);
    HIP_TRY(hipSetDevice(device));
    fskmc_ctx* c = new fskmc_ctx();
    c->device = device;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete c;
            return fail(FSKMC_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        c->own_stream = true;
    }
    if (hipMalloc((void**)&c->d_obs, 16 * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc((void**)&c->h_obs, 16 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->stage_free, hipEventDisableTiming) != hipSuccess ||
        hipMalloc((void**)&c->d_abort, sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void**)&c->d_queue, sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc((void**)&c->h_abort, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        fskmc_ctx_destroy(c);
        return fail(FSKMC_ENOMEM, "context allocation failed");
    }
    *c->h_abort = 0;
    if (launch_fill_u32(reinterpret_cast<uint32_t*>(c->d_abort), 1, 0u, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        fskmc_ctx_destroy(c);
        return fail(FSKMC_EDEVICE, "clearing the abort flag failed");
    }
    *out = c;
    return FSKMC_OK;
}

int fskmc_ctx_destroy(fskmc_ctx* c)
{
    if (!c)
        return FSKMC_OK;
    (void)hipSetDevice(c->device);
    if (c->stream)
        (void)hipStreamSynchronize(c->stream);
    // simulations still created on this context go with it
    for (fskmc_sim* S : c->sims.release_all()) {
        free_sim_device(S);
        delete S;
    }
    (void)hipFree(c->d_obs);
    (void)hipHostFree(c->h_obs);
    (void)hipFree(c->d_abort);
    (void)hipHostFree(c->h_abort);
    (void)hipFree(c->d_queue);
    if (c->graph_exec)
        (void)hipGraphExecDestroy(c->graph_exec);
    for (hipStream_t q : c->side) {
        (void)hipStreamSynchronize(q);
        (void)hipStreamDestroy(q);
    }
    if (c->upload) {
        (void)hipStreamSynchronize(c->upload);
        (void)hipStreamDestroy(c->upload);
    }
    for (hipEvent_t e : c->side_join)
        (void)hipEventDestroy(e);
    if (c->side_fork)
        (void)hipEventDestroy(c->side_fork);
    (void)hipFree(c->d_jobs);
    (void)hipFree(c->d_items);
    (void)hipHostFree(c->h_stage);
    if (c->stage_free)
        (void)hipEventDestroy(c->stage_free);
    for (hipEvent_t e : c->ev_pool)
        (void)hipEventDestroy(e);
    if (c->own_stream && c->stream)
        (void)hipStreamDestroy(c->stream);
    delete c;
    return FSKMC_OK;
}

int fskmc_ctx_set_batch_streams(fskmc_ctx* c, int streams)
{
    if (!c)
        return fail(FSKMC_EINVAL, "ctx is NULL");
    if (streams < 1 || streams > 4)
        return fail(FSKMC_EINVAL, "streams must be 1..4");
    c->batch_streams = streams;
    return FSKMC_OK;
}

int fskmc_ctx_set_batch_persistent(fskmc_ctx* c, int windows)
{
    if (!c)
        return fail(FSKMC_EINVAL, "ctx is NULL");
    if (windows < 0)
        return fail(FSKMC_EINVAL, "windows must be >= 0");
    c->batch_persist = (uint32_t)windows;
    return FSKMC_OK;
}

int fskmc_ctx_set_graphs(fskmc_ctx* c, int on)
{
    if (!c)
        return fail(FSKMC_EINVAL, "ctx is NULL");
    c->graphs = on != 0;
    return FSKMC_OK;
}

int fskmc_ctx_set_persistent(fskmc_ctx* c, int windows)
{
    if (!c)
        return fail(FSKMC_EINVAL, "ctx is NULL");
    if (windows < 0)
        return fail(FSKMC_EINVAL, "windows must be >= 0");
    c->persist = windows;
    return FSKMC_OK;
}

int fskmc_ctx_set_wait_limit(fskmc_ctx* c, double seconds)
{
    if (!c)
        return fail(FSKMC_EINVAL, "ctx is NULL");
    if (!(seconds > 0.0) || !(seconds <= 60.0))
        return fail(FSKMC_EINVAL, "wait limit must be in (0, 60] seconds");
    const double ticks = seconds * 1e8;
    c->wait_ticks = ticks < 1.0 ? 1ull : (unsigned long long)ticks;
    return FSKMC_OK;
}

int fskmc_ctx_set_rebalance(fskmc_ctx* c, int on)
{
    if (!c)
        return fail(FSKMC_EINVAL, "ctx is NULL");
    c->rebalance = on != 0;
    return FSKMC_OK;
}

int fskmc_workload_partition(const uint64_t* W, int M, int P, int cap, int32_t* bounds)
{
    if (M < 0 || P < 1 || cap < 0 || (M > 0 && !W) || !bounds)
        return fail(FSKMC_EINVAL, "need M >= 0, P >= 1, cap >= 0 and non-NULL arrays");
    if (cap > 0 && (int64_t)M > (int64_t)P * cap)
        return fail(FSKMC_EINVAL, "%d blocks do not fit %d processors of capacity %d", M, P, cap);
    cdf_ranges(W, M, P, cap, bounds);
    return FSKMC_OK;
}

int fskmc_sim_workload(fskmc_sim* S, uint64_t* out, size_t n_blocks)
{
    if (!S || !out)
        return fail(FSKMC_EINVAL, "NULL argument");
    if (n_blocks != (size_t)S->nb)
        return fail(FSKMC_EINVAL, "sim has %d blocks, got %zu", S->nb, n_blocks);
    if (int rc = check_valid(S))
        return rc;
    std::vector<BlockCount> rec(n_blocks);
    HIP_TRY(hipMemcpyAsync(rec.data(), S->d_cnt, n_blocks * sizeof(BlockCount), hipMemcpyDeviceToHost,
                           S->ctx->stream));
    HIP_TRY(hipStreamSynchronize(S->ctx->stream));
    for (size_t i = 0; i < n_blocks; ++i)
        out[i] = rec[i].events;
    return check_abort(S->ctx);
}

int fskmc_sim_last_partition(const fskmc_sim* S, int32_t* out, size_t n, size_t* n_out)
{
    if (!S || !n_out || (n > 0 && !out))
        return fail(FSKMC_EINVAL, "NULL argument");
    *n_out = S->n_owner;
    if (S->n_owner == 0 || n == 0) // n == 0: size query
        return FSKMC_OK;
    if (n < S->n_owner)
        return fail(FSKMC_EINVAL, "need room for %zu boundaries", S->n_owner);
    HIP_TRY(hipMemcpyAsync(out, S->d_owner, S->n_owner * 4, hipMemcpyDeviceToHost, S->ctx->stream));
    HIP_TRY(hipStreamSynchronize(S->ctx->stream));
    return check_abort(S->ctx);
}

int fskmc_ctx_set_resident(fskmc_ctx* c, int on)
{
    if (!c)
        return fail(FSKMC_EINVAL, "ctx is NULL");
    c->resident = on != 0;
    return FSKMC_OK;
}

int fskmc_ctx_set_nested(fskmc_ctx* c, int on)
{
    if (!c)
        return fail(FSKMC_EINVAL, "ctx is NULL");
    c->nested_kernel = on != 0;
    return FSKMC_OK;
}

int fskmc_ctx_set_kernel_timing(fskmc_ctx* c, int stride)
{
    if (!c)
        return fail(FSKMC_EINVAL, "ctx is NULL");
    if (stride < 0)
        return fail(FSKMC_EINVAL, "stride must be >= 0");
    c->timing_stride = stride;
    c->launch_counter = 0;
    return FSKMC_OK;
}

int fskmc_ctx_read_kernel_timing(fskmc_ctx* c, double* total_ms, uint64_t* n_launches)
{
    if (!c || !total_ms || !n_launches)
        return fail(FSKMC_EINVAL, "NULL argument");
    int rc = harvest_timing(c);
    if (rc)
        return rc;
    *total_ms = c->timed_ms;
    *n_launches = c->timed_n;
    c->timed_ms = 0.0;
    c->timed_n = 0;
    return FSKMC_OK;
}

int fskmc_ctx_set_waves_per_group(fskmc_ctx* c, int waves)
{
    if (!c)
        return fail(FSKMC_EINVAL, "ctx is NULL");
    if (waves != 1 && waves != 2 && waves != 4 && waves != 8)
        return fail(FSKMC_EINVAL, "waves per group must be 1, 2, 4 or 8");
    c->wpg = waves;
    return FSKMC_OK;
}

int fskmc_sync(fskmc_ctx* c)
{
    if (!c)
        return fail(FSKMC_EINVAL, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream));
    return check_abort(c);
}

// Independence of the coarse cells of one outer colour, as blocks of
// (cx bx) x (cy by) sites (eq. opdecomp at the coarse level): the nested
// scheme evolves them independently with their rings frozen.
int check_coarse(const fskmc_sim& S)
{
    if (S.NCX < 2 || S.NCY < 2)
        return fail(FSKMC_EDECOMP, "the nested decomposition needs at least 2 x 2 coarse cells (got %d x %d)", S.NCX,
                    S.NCY);
    fskmc_sim C;
    C.lat = S.lat;
    C.model = S.model;
    C.bx = S.bx * S.cx;
    C.by = S.by * S.cy;
    C.NBX = S.NCX;
    C.NBY = S.NCY;
    C.nb = S.NCX * S.NCY;
    C.n_colours = S.k_outer;
    C.blocks = S.cells;
    C.colour_off = S.cell_off;
    const int rc = check_decomposition(C);
    return rc ? fail(rc, "coarse cells of one outer colour interact: %s", fskmc_last_error()) : FSKMC_OK;
}

// The model's parameters into prm[0..4] (spin flip: k_a, k_d, J, h, beta;
// reaction model: y, k_r, D; spin exchange: D, J, beta), checked.
int parse_params(int model, const void* params, double prm[5])
{
    for (int i = 0; i < 5; ++i)
        prm[i] = 0.0;
    if (model == FSKMC_MODEL_FLIP) {
        const fskmc_flip_params* p = (const fskmc_flip_params*)params;
        double v[5] = {p->k_a, p->k_d, p->J, p->h, p->beta};
        for (int i = 0; i < 5; ++i)
            prm[i] = v[i];
        if (!(p->k_a >= 0) || !(p->k_d >= 0) || !std::isfinite(p->J) || !std::isfinite(p->h) ||
            !std::isfinite(p->beta) || !std::isfinite(p->k_a) || !std::isfinite(p->k_d))
            return fail(FSKMC_EINVAL, "spin-flip rates must be finite and k_a, k_d >= 0");
    } else if (model == FSKMC_MODEL_KAWASAKI) {
        const fskmc_kawasaki_params* p = (const fskmc_kawasaki_params*)params;
        prm[0] = p->D;
        prm[1] = p->J;
        prm[2] = p->beta;
        if (!(p->D >= 0) || !std::isfinite(p->D) || !std::isfinite(p->J) || !std::isfinite(p->beta))
            return fail(FSKMC_EINVAL, "spin exchange needs D >= 0 and finite D, J, beta");
    } else {
        const fskmc_zgb_params* p = (const fskmc_zgb_params*)params;
        prm[0] = p->y;
        prm[1] = p->k_r;
        prm[2] = p->D;
        if (!(p->y >= 0 && p->y <= 1) || !(p->k_r >= 0) || !(p->D >= 0) || !std::isfinite(p->k_r) ||
            !std::isfinite(p->D))
            return fail(FSKMC_EINVAL, "reaction model needs 0 <= y <= 1, k_r >= 0, D >= 0");
    }
    return FSKMC_OK;
}

int sim_create(fskmc_ctx* ctx, const fskmc_lattice* lattice, int model, const void* params,
               const fskmc_decomp* decomp, const fskmc_schedule* schedule, fskmc_key key, const fskmc_nested* nest,
               fskmc_sim** out)
{
    if (!ctx || !out || !params || !decomp || !schedule)
        return fail(FSKMC_EINVAL, "NULL argument");
    *out = nullptr;
    int rc = validate_lattice(lattice);
    if (rc)
        return rc;
    if (model != FSKMC_MODEL_FLIP && model != FSKMC_MODEL_ZGB && model != FSKMC_MODEL_KAWASAKI)
        return fail(FSKMC_EINVAL, "unknown model %d", model);
    fskmc_sim* S = new fskmc_sim();
    S->ctx = ctx;
    S->model = model;
    S->lat = *lattice;
    if ((rc = parse_params(model, params, S->prm))) {
        delete S;
        return rc;
    }
    S->bx = decomp->bx;
    S->by = decomp->by;
    S->n_colours = decomp->n_colours;
    S->sched = *schedule;
    S->key = key;
    if (S->bx <= 0 || S->by <= 0 || S->lat.Lx % S->bx || S->lat.Ly % S->by) {
        delete S;
        return fail(FSKMC_EINVAL, "blocks %dx%d do not tile %dx%d", decomp->bx, decomp->by, lattice->Lx, lattice->Ly);
    }
    if ((rc = kernel_shape(S->lat, model, S->bx, S->by, &S->P, &S->shape))) {
        delete S;
        return rc;
    }
    S->NBX = S->lat.Lx / S->bx;
    S->NBY = S->lat.Ly / S->by;
    S->nb = S->NBX * S->NBY;
    if (S->n_colours < 1 || S->n_colours > 127) {
        delete S;
        return fail(FSKMC_EINVAL, "n_colours must be in [1,127]");
    }
    if (nest) {
        S->nested = true;
        S->cx = nest->cx;
        S->cy = nest->cy;
        S->k_outer = nest->outer_colours;
        S->k_inner = nest->inner_colours;
        S->inner_split = nest->inner_split;
        S->dtau = nest->dtau;
        if (S->lat.dim != 2 || S->cx < 1 || S->cy < 1 || S->NBX % S->cx || S->NBY % S->cy) {
            delete S;
            return fail(FSKMC_EINVAL, "coarse cells of %dx%d blocks do not tile the %dx%d block grid", nest->cx,
                        nest->cy, S->NBX, S->NBY);
        }
        if ((S->k_outer != 2 && S->k_outer != 4) || (S->k_inner != 2 && S->k_inner != 4)) {
            delete S;
            return fail(FSKMC_EINVAL, "outer and inner colourings have 2 or 4 colours");
        }
        S->NCX = S->NBX / S->cx;
        S->NCY = S->NBY / S->cy;
        auto builtin = [](int k, int i, int j) { return k == 2 ? (i + j) % 2 : (i % 2) + 2 * (j % 2); };
        S->cell_off.assign(S->k_outer + 1, 0);
        for (int c = 0; c < S->k_outer; ++c) {
            S->cell_off[c] = (int32_t)S->cells.size();
            for (int q = 0; q < S->NCX * S->NCY; ++q)
                if (builtin(S->k_outer, q % S->NCX, q / S->NCX) == c)
                    S->cells.push_back(q);
        }
        S->cell_off[S->k_outer] = (int32_t)S->cells.size();
        S->cmap.resize(S->nb);
        for (int m = 0; m < S->nb; ++m) {
            const int bi = m % S->NBX, bj = m / S->NBX;
            S->cmap[m] = builtin(S->k_outer, bi / S->cx, bj / S->cy) * S->k_inner +
                         builtin(S->k_inner, bi % S->cx, bj % S->cy);
        }
        if ((rc = check_coarse(*S))) {
            delete S;
            return rc;
        }
        S->nest_kernel_ok = S->cx == S->cy && nested_supported(kernel_model(model), S->P, S->cx, S->k_inner);
    }
    S->cmap.resize(S->nb);
    for (int m = 0; m < S->nb && !nest; ++m) {
        const int bi = m % S->NBX, bj = m / S->NBX;
        int c;
        if (decomp->colour_map) {
            c = decomp->colour_map[m];
        } else if (S->n_colours == 2) {
            c = (bi + bj) % 2;
        } else if (S->n_colours == 4) {
            c = (bi % 2) + 2 * (bj % 2);
        } else {
            delete S;
            return fail(FSKMC_EINVAL, "built-in colour maps have 2 or 4 colours");
        }
        if (c < 0 || c >= S->n_colours) {
            delete S;
            return fail(FSKMC_EINVAL, "colour_map[%d] = %d out of range", m, c);
        }
        S->cmap[m] = c;
    }
    S->colour_off.assign(S->n_colours + 1, 0);
    for (int c = 0; c < S->n_colours; ++c) {
        S->colour_off[c] = (int32_t)S->blocks.size();
        for (int m = 0; m < S->nb; ++m)
            if (S->cmap[m] == c)
                S->blocks.push_back(m);
        S->max_per_colour = std::max(S->max_per_colour, (int)S->blocks.size() - S->colour_off[c]);
    }
    S->colour_off[S->n_colours] = (int32_t)S->blocks.size();
    if ((rc = check_decomposition(*S)) || (rc = nest ? build_nested_schedule(*S) : build_schedule(*S))) {
        delete S;
        return rc;
    }
    build_table(*S);
    if ((rc = check_table(S->table.data(), (int)S->table.size()))) {
        delete S;
        return rc;
    }
    // persistent-sweep tables: next window of each colour, colour per block,
    // interacting blocks
    const size_t nw1 = (size_t)S->n_windows + 1;
    S->next_part.assign((size_t)S->n_colours * nw1, (int32_t)S->n_windows);
    for (int c = 0; c < S->n_colours; ++c)
        for (int64_t w = (int64_t)S->n_windows - 1; w >= 0; --w)
            S->next_part[c * nw1 + w] = S->win_colour[w] == c ? (int32_t)w : S->next_part[c * nw1 + w + 1];
    std::vector<int8_t> bcol(S->cmap.begin(), S->cmap.end());
    std::vector<int32_t> nbr;
    build_neighbours(*S, nbr);
    (void)hipSetDevice(ctx->device);
    const int64_t N = n_sites(S->lat);
    if ((rc = dev_alloc(&S->d_lat, (size_t)N)) || (rc = dev_alloc(&S->d_table, S->table.size())) ||
        (rc = dev_alloc(&S->d_cnt, S->nb)) || (rc = dev_alloc(&S->d_blocks, S->blocks.size())) ||
        (rc = dev_alloc(&S->d_coff, S->colour_off.size())) ||
        // padded to whole dwords: the resident sweep reads a window's colour
        // with a scalar dword load
        (rc = dev_alloc(&S->d_wcol, (S->n_windows + 3) & ~(size_t)3)) ||
        (rc = dev_alloc(&S->d_wdur, S->n_windows)) || (rc = dev_alloc(&S->d_bcol, S->nb)) ||
        (rc = dev_alloc(&S->d_next, S->next_part.size())) || (rc = dev_alloc(&S->d_nbr, nbr.size())) ||
        (rc = dev_alloc(&S->d_epoch, S->nb)) ||
        (rc = dev_alloc(&S->d_edge, 4 * (size_t)S->nb)) || (rc = dev_alloc(&S->d_cells, S->cells.size())) ||
        (rc = dev_alloc(&S->d_ofirst, S->ofirst.size()))) {
        free_sim_device(S);
        delete S;
        return rc;
    }
    // the uploads and the zeroed lattice go through the context's upload
    // stream and only that stream is waited for: work already queued on the
    // context's stream (a running batch) keeps the GPU busy meanwhile
    hipError_t e = hipSuccess;
    if (!ctx->upload)
        e = hipStreamCreateWithFlags(&ctx->upload, hipStreamNonBlocking);
    hipStream_t st = ctx->upload;
    if (e == hipSuccess)
        e = hipMemcpyAsync(S->d_bcol, bcol.data(), bcol.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !S->cells.empty())
        e = hipMemcpyAsync(S->d_cells, S->cells.data(), S->cells.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !S->ofirst.empty())
        e = hipMemcpyAsync(S->d_ofirst, S->ofirst.data(), S->ofirst.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(S->d_next, S->next_part.data(), S->next_part.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(S->d_nbr, nbr.data(), nbr.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(S->d_table, S->table.data(), S->table.size() * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(S->d_blocks, S->blocks.data(), S->blocks.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(S->d_coff, S->colour_off.data(), S->colour_off.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && S->n_windows)
        e = hipMemcpyAsync(S->d_wcol, S->win_colour.data(), S->n_windows, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && S->n_windows)
        e = hipMemcpyAsync(S->d_wdur, S->win_dur.data(), S->n_windows * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_init(S->d_lat, N, 0, 0.0, 0, 0, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st); // the host vectors above are pageable
    if (e != hipSuccess || (rc = reset_counters(S))) {
        free_sim_device(S);
        delete S;
        return e != hipSuccess ? fail(FSKMC_EDEVICE, "sim upload failed: %s", hipGetErrorString(e)) : rc;
    }
    ctx->sims.add(S);
    *out = S;
    return FSKMC_OK;
}

int fskmc_sim_create(fskmc_ctx* ctx, const fskmc_lattice* lattice, int model, const void* params,
                     const fskmc_decomp* decomp, const fskmc_schedule* schedule, fskmc_key key, fskmc_sim** out)
{
    return sim_create(ctx, lattice, model, params, decomp, schedule, key, nullptr, out);
}

int fskmc_sim_create_nested(fskmc_ctx* ctx, const fskmc_lattice* lattice, int model, const void* params,
                            const fskmc_nested* nested, const fskmc_schedule* schedule, fskmc_key key,
                            fskmc_sim** out)
{
    if (!nested)
        return fail(FSKMC_EINVAL, "NULL argument");
    const fskmc_decomp d{nested->bx, nested->by, nested->outer_colours * nested->inner_colours, nullptr};
    return sim_create(ctx, lattice, model, params, &d, schedule, key, nested, out);
}

int fskmc_sim_destroy(fskmc_sim* S)
{
    if (!S)
        return FSKMC_OK;
    (void)hipSetDevice(S->ctx->device);
    (void)hipStreamSynchronize(S->ctx->stream);
    S->ctx->sims.remove(S);
    free_sim_device(S);
    delete S;
    return FSKMC_OK;
}

int fskmc_sim_attach_device_lattice(fskmc_sim* S, void* dev_ptr, size_t bytes)
{
    if (!S || !dev_ptr)
        return fail(FSKMC_EINVAL, "NULL argument");
    const size_t N = (size_t)n_sites(S->lat);
    if (bytes < N)
        return fail(FSKMC_EINVAL, "buffer of %zu bytes, lattice needs %zu", bytes, N);
    if (((uintptr_t)dev_ptr) % 16)
        return fail(FSKMC_EINVAL, "device lattice must be 16-byte aligned");
    if (dev_ptr == S->d_lat)
        return FSKMC_OK;
    HIP_TRY(hipMemcpyAsync(dev_ptr, S->d_lat, N, hipMemcpyDeviceToDevice, S->ctx->stream));
    HIP_TRY(hipStreamSynchronize(S->ctx->stream));
    if (S->own_lat)
        HIP_TRY(hipFree(S->d_lat));
    S->d_lat = (uint8_t*)dev_ptr;
    S->own_lat = false;
    return FSKMC_OK;
}

int fskmc_sim_init(fskmc_sim* S, int kind, double p)
{
    if (!S)
        return fail(FSKMC_EINVAL, "sim is NULL");
    if (kind != 0 && kind != 1)
        return fail(FSKMC_EINVAL, "init kind must be 0 (empty) or 1 (Bernoulli)");
    if (kind == 1 && !(p >= 0.0 && p <= 1.0))
        return fail(FSKMC_EINVAL, "Bernoulli p must be in [0,1]");
    HIP_TRY(launch_init(S->d_lat, n_sites(S->lat), kind, p, S->key.seed, S->key.replica, S->ctx->stream));
    S->window = 0;
    S->invalid = false;
    return reset_counters(S);
}

int fskmc_sim_set_lattice(fskmc_sim* S, const uint8_t* host, size_t n)
{
    if (!S || !host)
        return fail(FSKMC_EINVAL, "NULL argument");
    if (n != (size_t)n_sites(S->lat))
        return fail(FSKMC_EINVAL, "lattice has %lld sites, got %zu bytes", (long long)n_sites(S->lat), n);
    const int K = S->model == FSKMC_MODEL_ZGB ? 3 : 2;
    for (size_t i = 0; i < n; ++i)
        if (host[i] >= K)
            return fail(FSKMC_EINVAL, "site %zu has state %d outside [0,%d)", i, (int)host[i], K);
    HIP_TRY(hipMemcpyAsync(S->d_lat, host, n, hipMemcpyHostToDevice, S->ctx->stream));
    HIP_TRY(hipStreamSynchronize(S->ctx->stream));
    return FSKMC_OK;
}

int fskmc_sim_get_lattice(fskmc_sim* S, uint8_t* host, size_t n)
{
    if (!S || !host)
        return fail(FSKMC_EINVAL, "NULL argument");
    if (n != (size_t)n_sites(S->lat))
        return fail(FSKMC_EINVAL, "lattice has %lld sites, got %zu bytes", (long long)n_sites(S->lat), n);
    if (int rc = check_valid(S))
        return rc;
    HIP_TRY(hipMemcpyAsync(host, S->d_lat, n, hipMemcpyDeviceToHost, S->ctx->stream));
    HIP_TRY(hipStreamSynchronize(S->ctx->stream));
    return check_abort(S->ctx);
}

int fskmc_sim_advance(fskmc_sim* S, uint64_t n_windows)
{
    if (!S)
        return fail(FSKMC_EINVAL, "sim is NULL");
    if (int rc = check_valid(S))
        return rc;
    if (n_windows > S->n_windows - S->window)
        return fail(FSKMC_ESTATE, "only %llu windows left before T", (unsigned long long)(S->n_windows - S->window));
    if (S->nested && S->nest_kernel_ok && S->ctx->nested_kernel) {
        const uint64_t end = S->window + n_windows;
        fskmc_ctx* c = S->ctx;
        bool resident = c->persist > 0 && c->resident && S->model == FSKMC_MODEL_FLIP && S->nest_resident_fits;
        while (S->window < end) {
            if (resident) {
                const uint64_t w1 = std::min<uint64_t>(end, S->window + (uint64_t)c->persist);
                const int rc = enqueue_nested_resident(S, S->window, w1);
                if (rc == FSKMC_OK) {
                    S->window = w1;
                    continue;
                }
                if (rc != 1)
                    return rc;
                S->nest_resident_fits = resident = false;
            }
            const uint64_t w1 = std::min<uint64_t>(end, S->outer_end[S->window]);
            if (int rc = enqueue_nested(S, S->window, w1))
                return rc;
            S->window = w1;
        }
        return FSKMC_OK;
    }
    if (S->ctx->persist > 0) {
        uint64_t left = n_windows;
        while (left > 0) {
            const uint64_t k = std::min<uint64_t>(left, (uint64_t)S->ctx->persist);
            int rc = 1;
            if (S->ctx->resident && S->model == FSKMC_MODEL_FLIP)
                rc = enqueue_resident(S, S->window, S->window + k);
            if (rc == 1)
                rc = enqueue_persistent(S, S->window, S->window + k);
            if (rc)
                return rc;
            S->window += k;
            left -= k;
        }
        return FSKMC_OK;
    }
    for (uint64_t i = 0; i < n_windows; ++i) {
        int rc = enqueue_window(S, S->window);
        if (rc)
            return rc;
        S->window++;
    }
    return FSKMC_OK;
}

int fskmc_sim_run_to_end(fskmc_sim* S)
{
    if (!S)
        return fail(FSKMC_EINVAL, "sim is NULL");
    return fskmc_sim_advance(S, S->n_windows - S->window);
}

int fskmc_sim_windows(const fskmc_sim* S, uint64_t* total, uint64_t* next)
{
    if (!S)
        return fail(FSKMC_EINVAL, "sim is NULL");
    if (total)
        *total = S->n_windows;
    if (next)
        *next = S->window;
    return FSKMC_OK;
}

int fskmc_sim_observe(fskmc_sim* S, fskmc_obs* out)
{
    if (!S || !out)
        return fail(FSKMC_EINVAL, "NULL argument");
    if (int rc = check_valid(S))
        return rc;
    fskmc_ctx* c = S->ctx;
    HIP_TRY(launch_fill_u64((uint64_t*)c->d_obs, 9, 0ull, c->stream));
    HIP_TRY(launch_observe(S->d_lat, S->lat.Lx, S->lat.Ly, S->lat.dim, S->d_cnt, S->nb, c->d_obs,
                           c->stream));
    HIP_TRY(hipMemcpyAsync(c->h_obs, c->d_obs, 9 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (int rc = check_abort(c))
        return rc;
    std::memset(out, 0, sizeof *out);
    out->n_sites = n_sites(S->lat);
    for (int k = 0; k < 3; ++k) {
        out->count[k] = (int64_t)c->h_obs[k];
        out->bonds_equal[k] = (int64_t)c->h_obs[3 + k];
    }
    out->bonds_ab = (int64_t)c->h_obs[6];
    out->events = c->h_obs[7];
    out->writes = c->h_obs[8];
    out->block_windows = S->block_windows;
    out->window = S->window;
    uint64_t steps = 0;
    for (uint64_t w = 0; w < S->window; ++w)
        steps += S->step_end[w];
    out->steps = steps;
    out->t = (double)steps * S->sched.dt;
    return FSKMC_OK;
}

int fskmc_sim_block_events(fskmc_sim* S, uint32_t* out, size_t n_blocks)
{
    if (!S || !out)
        return fail(FSKMC_EINVAL, "NULL argument");
    if (n_blocks != (size_t)S->nb)
        return fail(FSKMC_EINVAL, "sim has %d blocks, got %zu", S->nb, n_blocks);
    if (int rc = check_valid(S))
        return rc;
    std::vector<BlockCount> rec(n_blocks);
    HIP_TRY(hipMemcpyAsync(rec.data(), S->d_cnt, n_blocks * sizeof(BlockCount), hipMemcpyDeviceToHost,
                           S->ctx->stream));
    HIP_TRY(hipStreamSynchronize(S->ctx->stream));
    for (size_t i = 0; i < n_blocks; ++i)
        out[i] = rec[i].W;
    return check_abort(S->ctx);
}

int fskmc_sim_rate_table(const fskmc_sim* S, double* out, size_t n)
{
    if (!S || !out)
        return fail(FSKMC_EINVAL, "NULL argument");
    if (n < S->table.size())
        return fail(FSKMC_EINVAL, "table has %zu entries", S->table.size());
    std::memcpy(out, S->table.data(), S->table.size() * 8);
    return (int)S->table.size();
}

int fskmc_sim_get_state(fskmc_sim* S, uint64_t* window, uint8_t* host, size_t n)
{
    if (!S || !window || !host)
        return fail(FSKMC_EINVAL, "NULL argument");
    int rc = fskmc_sim_get_lattice(S, host, n);
    if (rc)
        return rc;
    *window = S->window;
    return FSKMC_OK;
}

int fskmc_sim_set_state(fskmc_sim* S, uint64_t window, const uint8_t* host, size_t n)
{
    if (!S || !host)
        return fail(FSKMC_EINVAL, "NULL argument");
    if (window > S->n_windows)
        return fail(FSKMC_EINVAL, "window %llu beyond the schedule (%llu)", (unsigned long long)window,
                    (unsigned long long)S->n_windows);
    int rc = fskmc_sim_set_lattice(S, host, n);
    if (rc)
        return rc;
    S->window = window;
    S->invalid = false;
    return reset_counters(S);
}

size_t fskmc_sim_footprint(const fskmc_lattice* lattice, int model, const fskmc_decomp* decomp,
                           const fskmc_schedule* schedule)
{
    if (!lattice || !decomp || !schedule || lattice->Lx <= 0 || lattice->Ly <= 0 || decomp->bx <= 0 ||
        decomp->by <= 0 || !(schedule->dt > 0))
        return 0;
    const int64_t N = (int64_t)lattice->Lx * lattice->Ly;
    const int nb = (lattice->Lx / decomp->bx) * (lattice->Ly / decomp->by);
    const int K = decomp->n_colours;
    const uint64_t per = schedule->split == FSKMC_STRANG ? 2 * K - 1 : K;
    const uint64_t nw = (uint64_t)std::floor(schedule->T / schedule->dt + 0.5) * per;
    return footprint_of(N, model, nb, nw, K);
}

// At least n - 1 side streams (default priority) and their join events, plus
// the fork event, created on the context's device.
static int ensure_side_streams(fskmc_ctx* ctx, int n)
{
    if ((int)ctx->side.size() >= n - 1 && ctx->side_fork)
        return FSKMC_OK;
    int prev = 0;
    HIP_TRY(hipGetDevice(&prev));
    HIP_TRY(hipSetDevice(ctx->device));
    hipError_t e = hipSuccess;
    if (!ctx->side_fork)
        e = hipEventCreateWithFlags(&ctx->side_fork, hipEventDisableTiming);
    while (e == hipSuccess && (int)ctx->side.size() < n - 1) {
        hipStream_t q = nullptr;
        hipEvent_t j = nullptr;
        e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);
        if (e != hipSuccess)
            break;
        e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(q);
            break;
        }
        ctx->side.push_back(q);
        ctx->side_join.push_back(j);
    }
    (void)hipSetDevice(prev);
    if (e != hipSuccess)
        return fail(FSKMC_EDEVICE, "side streams: %s", hipGetErrorString(e));
    return FSKMC_OK;
}

int fskmc_batch_advance(fskmc_ctx* ctx, fskmc_sim* const* sims, int n, uint32_t windows)
{
    if (!ctx || (n > 0 && !sims) || n < 0)
        return fail(FSKMC_EINVAL, "bad arguments");
    if (n == 0 || windows == 0)
        return FSKMC_OK;
    for (int i = 0; i < n; ++i) {
        if (!sims[i] || sims[i]->ctx != ctx)
            return fail(FSKMC_EINVAL, "sim %d is NULL or belongs to another context", i);
        if (int rc = check_valid(sims[i]))
            return rc;
        for (int j = 0; j < i; ++j)
            if (sims[j] == sims[i])
                return fail(FSKMC_EINVAL, "sim %d appears twice", i);
    }
    // group the sims by kernel variant; each group is one launch per step
    struct Group {
        int model, P, shape;
        std::vector<int> idx;
        uint32_t items = 0;
        size_t job_off = 0, item_off = 0;
    };
    std::vector<Group> groups;
    for (int i = 0; i < n; ++i) {
        fskmc_sim* S = sims[i];
        if (S->window >= S->n_windows)
            continue;
        Group* g = nullptr;
        for (auto& gg : groups)
            if (gg.model == kernel_model(S->model) && gg.P == S->P && gg.shape == S->shape)
                g = &gg;
        if (!g) {
            groups.push_back(Group{kernel_model(S->model), S->P, S->shape, {}, 0, 0, 0});
            g = &groups.back();
        }
        g->idx.push_back(i);
    }
    size_t n_jobs = 0, n_items = 0;
    for (auto& g : groups) {
        g.job_off = n_jobs;
        g.item_off = n_items;
        for (int i : g.idx)
            g.items += (uint32_t)sims[i]->max_per_colour;
        n_jobs += g.idx.size();
        n_items += g.items;
    }
    if (n_jobs == 0)
        return FSKMC_OK;
    if (n_jobs > ctx->cap_jobs) {
        (void)hipFree(ctx->d_jobs);
        ctx->d_jobs = nullptr;
        ctx->cap_jobs = 0;
        int rc = dev_alloc(&ctx->d_jobs, n_jobs * 2);
        if (rc)
            return rc;
        ctx->cap_jobs = n_jobs * 2;
    }
    if (n_items > ctx->cap_items) {
        (void)hipFree(ctx->d_items);
        ctx->d_items = nullptr;
        ctx->cap_items = 0;
        int rc = dev_alloc(&ctx->d_items, n_items * 2);
        if (rc)
            return rc;
        ctx->cap_items = n_items * 2;
    }
    const size_t bytes = n_jobs * sizeof(JobDesc) + n_items * 4;
    HIP_TRY(hipEventSynchronize(ctx->stage_free)); // previous upload has left the staging buffer
    if (bytes > ctx->cap_stage) {
        (void)hipHostFree(ctx->h_stage);
        ctx->h_stage = nullptr;
        ctx->cap_stage = 0;
        if (hipHostMalloc((void**)&ctx->h_stage, bytes * 2, hipHostMallocDefault) != hipSuccess)
            return fail(FSKMC_ENOMEM, "pinned staging of %zu bytes failed", bytes * 2);
        ctx->cap_stage = bytes * 2;
    }
    JobDesc* hj = (JobDesc*)ctx->h_stage;
    uint32_t* hi = (uint32_t*)(ctx->h_stage + n_jobs * sizeof(JobDesc));
    for (auto& g : groups) {
        uint32_t item = 0;
        for (size_t k = 0; k < g.idx.size(); ++k) {
            fskmc_sim* S = sims[g.idx[k]];
            JobDesc& d = hj[g.job_off + k];
            d.lat = S->d_lat;
            d.table = S->d_table;
            d.cnt = S->d_cnt;
            d.blocks = S->d_blocks;
            d.colour_off = S->d_coff;
            d.win_colour = S->d_wcol;
            d.win_dur = S->d_wdur;
            d.n_windows = S->n_windows;
            d.base_window = S->window;
            d.Lx = S->lat.Lx;
            d.Ly = S->lat.Ly;
            d.NBX = S->NBX;
            d.k0 = S->key.seed;
            d.k1 = S->key.replica;
            d.item_begin = item;
            d.n_items = (uint32_t)S->max_per_colour;
            d.pad = 0;
            d.bcol = S->d_bcol;
            d.next_part = S->d_next;
            d.nbr = S->d_nbr;
            d.epoch = S->d_epoch;
            d.nb = S->nb;
            d.pad2 = 0;
            for (int q = 0; q < S->max_per_colour; ++q)
                hi[g.item_off + item + q] = (uint32_t)k;
            item += (uint32_t)S->max_per_colour;
        }
    }
    HIP_TRY(hipMemcpyAsync(ctx->d_jobs, hj, n_jobs * sizeof(JobDesc), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->d_items, hi, n_items * 4, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipEventRecord(ctx->stage_free, ctx->stream));
    const uint32_t K = ctx->batch_persist;
    hipStream_t st = ctx->stream;
    // packed launches of different groups touch different sims: with several
    // groups they run on streams of their own (group i on stream i mod ns),
    // each group's windows in order on its stream, all joined back into the
    // context's stream before the call's later work.  Not while kernel timing
    // samples launches (the samples would overlap), and not in a captured
    // graph: a process took a host segmentation fault inside this call on its
    // first capture across the side streams, with no cause found in this
    // code, so graph capture keeps every launch on the context's stream.
    const bool use_graph = ctx->graphs && ctx->timing_stride == 0;
    const int ns = (K == 0 && ctx->timing_stride == 0 && !use_graph)
                       ? std::min<int>((int)groups.size(), ctx->batch_streams) : 1;
    if (ns > 1)
        if (int rc = ensure_side_streams(ctx, ns))
            return rc;
    // The launch sequence of this call: one packed launch per window and
    // group, or (K > 0) the epochs of every job, then per K windows and group
    // a cleared work counter and one persistent launch.  It reads the job
    // table through device pointers only, so a captured graph of it replays
    // for any later call with the same layout.
    auto enqueue = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        if (K == 0) {
            if (ns > 1) {
                e = hipEventRecord(ctx->side_fork, st);
                for (int q = 0; q + 1 < ns && e == hipSuccess; ++q)
                    e = hipStreamWaitEvent(ctx->side[q], ctx->side_fork, 0);
            }
            for (uint32_t step = 0; step < windows && e == hipSuccess; ++step)
                for (size_t gi = 0; gi < groups.size(); ++gi) {
                    const Group& g = groups[gi];
                    const int q = (int)(gi % (size_t)ns);
                    const LaunchTiming tk = timing_begin(ctx);
                    e = launch_sweep_batched(g.model, g.P, g.shape, ctx->wpg, ctx->d_jobs + g.job_off,
                                             ctx->d_items + g.item_off, g.items, step,
                                             q == 0 ? st : ctx->side[q - 1], tk);
                    timing_end(ctx, tk);
                    if (e != hipSuccess)
                        break;
                }
            // the join is enqueued even after a failed launch, so the
            // context's stream never runs ahead of a side stream
            for (int q = 0; q + 1 < ns; ++q) {
                const hipError_t r = hipEventRecord(ctx->side_join[q], ctx->side[q]);
                const hipError_t w = r == hipSuccess ? hipStreamWaitEvent(st, ctx->side_join[q], 0) : r;
                if (e == hipSuccess)
                    e = w;
            }
            return e;
        }
        e = launch_epoch_init_batched(ctx->d_jobs, (int)n_jobs, st);
        for (uint32_t s0 = 0; s0 < windows && e == hipSuccess; s0 += K) {
            const uint32_t s1 = std::min<uint32_t>(windows, s0 + K);
            for (auto& g : groups) {
                const unsigned grid = batched_persistent_grid(g.P, g.shape, ctx->wpg);
                const uint64_t total = (uint64_t)(s1 - s0) * g.items;
                const uint64_t per = total / ((uint64_t)grid * ctx->wpg * 8);
                BatchPersistArgs a{};
                a.jobs = ctx->d_jobs + g.job_off;
                a.item_job = ctx->d_items + g.item_off;
                a.n_items = g.items;
                a.s0 = s0;
                a.s1 = s1;
                a.chunk = (uint32_t)std::min<uint64_t>(16, std::max<uint64_t>(1, per));
                a.queue = ctx->d_queue;
                a.abort_flag = ctx->d_abort;
                a.wait_ticks = ctx->wait_ticks;
                e = launch_fill_u64(reinterpret_cast<uint64_t*>(ctx->d_queue), 1, 0ull, st);
                if (e != hipSuccess)
                    break;
                const LaunchTiming tk = timing_begin(ctx);
                e = launch_sweep_batched_persistent(g.model, g.P, g.shape, ctx->wpg, a, 0, st, tk);
                timing_end(ctx, tk);
                if (e != hipSuccess)
                    break;
            }
        }
        return e;
    };
    if (use_graph) {
        // everything the captured launches bake in, the wait limit included
        std::vector<uint64_t> key = {windows, K, (uint64_t)ctx->wpg, (uint64_t)(uintptr_t)ctx->d_jobs,
                                     (uint64_t)(uintptr_t)ctx->d_items, (uint64_t)(uintptr_t)st, n_jobs,
                                     (uint64_t)ctx->wait_ticks, (uint64_t)ns};
        for (auto& g : groups)
            key.insert(key.end(), {(uint64_t)g.model, (uint64_t)g.P, (uint64_t)g.shape, g.job_off, g.item_off,
                                   g.items, g.idx.size()});
        if (!ctx->graph_exec || key != ctx->graph_key) {
            if (ctx->graph_exec) {
                (void)hipGraphExecDestroy(ctx->graph_exec);
                ctx->graph_exec = nullptr;
            }
            HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            const hipError_t e = enqueue();
            hipGraph_t graph = nullptr;
            const hipError_t ee = hipStreamEndCapture(st, &graph);
            if (e != hipSuccess || ee != hipSuccess) {
                if (graph)
                    (void)hipGraphDestroy(graph);
                return fail(FSKMC_EDEVICE, "graph capture of the batched launches failed: %s",
                            hipGetErrorString(e != hipSuccess ? e : ee));
            }
            const hipError_t ie = hipGraphInstantiate(&ctx->graph_exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) {
                ctx->graph_exec = nullptr;
                return fail(FSKMC_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ie));
            }
            ctx->graph_key = key;
        }
        HIP_TRY(hipGraphLaunch(ctx->graph_exec, st));
    } else {
        HIP_TRY(enqueue());
    }
    if (K > 0)
        HIP_TRY(hipMemcpyAsync(ctx->h_abort, ctx->d_abort, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    for (int i = 0; i < n; ++i) {
        fskmc_sim* S = sims[i];
        if (K > 0 && S->window < S->n_windows)
            ctx->sims.touched(S);
        const uint64_t end = std::min<uint64_t>(S->n_windows, S->window + windows);
        for (uint64_t w = S->window; w < end; ++w) {
            const int c = S->win_colour[w];
            S->block_windows += (uint64_t)(S->colour_off[c + 1] - S->colour_off[c]);
        }
        S->window = end;
    }
    return FSKMC_OK;
}

int fskmc_advance_noalloc(int device, void* hip_stream, const fskmc_lattice* lattice, int model, const void* params,
                          const fskmc_decomp* decomp, const fskmc_schedule* schedule, fskmc_key key,
                          uint8_t* d_lattice, uint64_t w0, uint64_t n_windows, uint32_t* d_block_events,
                          unsigned long long* d_events)
{
    // everything is checked before the first HIP call
    if (!params || !decomp || !schedule || !d_lattice)
        return fail(FSKMC_EINVAL, "NULL argument");
    int rc = validate_lattice(lattice);
    if (rc)
        return rc;
    if (model != FSKMC_MODEL_FLIP && model != FSKMC_MODEL_ZGB && model != FSKMC_MODEL_KAWASAKI)
        return fail(FSKMC_EINVAL, "unknown model %d", model);
    double prm[5];
    if ((rc = parse_params(model, params, prm)))
        return rc;
    const int bx = decomp->bx, by = decomp->by, K = decomp->n_colours;
    if (bx <= 0 || by <= 0 || lattice->Lx % bx || lattice->Ly % by)
        return fail(FSKMC_EINVAL, "blocks %dx%d do not tile %dx%d", bx, by, lattice->Lx, lattice->Ly);
    int P = 0, shape = 0;
    if ((rc = kernel_shape(*lattice, model, bx, by, &P, &shape)))
        return rc;
    if (decomp->colour_map)
        return fail(FSKMC_EINVAL, "the allocation-free advance takes the built-in colour maps only");
    if (K != 2 && K != 4)
        return fail(FSKMC_EINVAL, "built-in colour maps have 2 or 4 colours");
    const int NBX = lattice->Lx / bx, NBY = lattice->Ly / by;
    const int64_t nb64 = (int64_t)NBX * NBY;
    if (nb64 > kNoallocMaxBlocks)
        return fail(FSKMC_EINVAL, "%lld blocks exceed the %d of the allocation-free advance's static scratch",
                    (long long)nb64, kNoallocMaxBlocks);
    const int nb = (int)nb64;
    // Independence of the built-in maps (Sec. 2.1), block by block: blocks are
    // at least 8 sites on a side, so a block's closure reaches only the blocks
    // next to it (spin flip: across a side; pair events: across a side or a
    // corner), and no two of those may share its colour.
    const bool pair = model != FSKMC_MODEL_FLIP;
    auto colour = [&](int bi, int bj) { return K == 2 ? (bi + bj) % 2 : (bi % 2) + 2 * (bj % 2); };
    int32_t count[4] = {0, 0, 0, 0};
    for (int bj = 0; bj < NBY; ++bj)
        for (int bi = 0; bi < NBX; ++bi) {
            const int c = colour(bi, bj);
            ++count[c];
            for (int dj = -1; dj <= 1; ++dj)
                for (int di = -1; di <= 1; ++di) {
                    if ((di == 0 && dj == 0) || (!pair && di != 0 && dj != 0) || (lattice->dim == 1 && dj != 0))
                        continue;
                    const int ni = (bi + di + NBX) % NBX, nj = (bj + dj + NBY) % NBY;
                    if ((ni != bi || nj != bj) && colour(ni, nj) == c)
                        return fail(FSKMC_EDECOMP, "blocks of colour %d interact (blocks %d and %d)", c,
                                    bj * NBX + bi, nj * NBX + ni);
                }
        }
    int64_t steps = 0;
    int per = 0;
    if ((rc = scheme_steps(schedule->split, K, schedule->dt, schedule->T, &steps, &per)))
        return rc;
    const uint64_t total = (uint64_t)steps * (uint64_t)per;
    if (w0 > total || n_windows > total - w0)
        return fail(FSKMC_ESTATE, "windows [%llu, %llu) are past the schedule's %llu",
                    (unsigned long long)w0, (unsigned long long)(w0 + n_windows), (unsigned long long)total);
    double tab[243 * 14];
    const int ntab = table_size(model, lattice->dim);
    fill_table(model, lattice->dim, prm, tab);
    if ((rc = check_table(tab, ntab)))
        return rc;
    int32_t off[4] = {0, 0, 0, 0};
    for (int c = 1; c < 4; ++c)
        off[c] = off[c - 1] + count[c - 1];

    int prev = 0;
    HIP_TRY(hipGetDevice(&prev));
    uint8_t* base = nullptr;
    hipError_t e = noalloc_scratch(device, &base);
    if (e != hipSuccess)
        return fail(FSKMC_EDEVICE, "scratch of device %d: %s", device, hipGetErrorString(e));
    HIP_TRY(hipSetDevice(device));
    hipStream_t st = (hipStream_t)hip_stream;
    double* d_tab = reinterpret_cast<double*>(base);
    int32_t* d_blocks = reinterpret_cast<int32_t*>(base + kNoallocBlocksOff);
    BlockCount* d_cnt = reinterpret_cast<BlockCount*>(base + kNoallocCountOff);
    // the previous call's contents are overwritten; counters start at zero
    e = launch_put_f64(d_tab, tab, ntab, st);
    if (e == hipSuccess)
        e = launch_builtin_blocks(d_blocks, NBX, NBY, K, off, st);
    if (e == hipSuccess)
        e = launch_fill_u64(reinterpret_cast<uint64_t*>(d_cnt), 2 * (int64_t)nb, 0ull, st);
    for (uint64_t w = w0; e == hipSuccess && w < w0 + n_windows; ++w) {
        int c = 0;
        double d = 0.0;
        scheme_window(schedule->split, K, schedule->dt, key, (int)(w % (uint64_t)per), (uint32_t)w, &c, &d);
        SweepArgs a;
        a.lat = d_lattice;
        a.table = d_tab;
        a.cnt = d_cnt;
        a.blocks = d_blocks + off[c];
        a.n_blocks = count[c];
        a.Lx = lattice->Lx;
        a.Ly = lattice->Ly;
        a.NBX = NBX;
        a.k0 = key.seed;
        a.k1 = key.replica;
        a.w = (uint32_t)w;
        a.dur = d;
        e = launch_sweep_single(kernel_model(model), P, shape, 2, a, st, LaunchTiming{});
    }
    if (e == hipSuccess && (d_block_events || d_events))
        e = launch_noalloc_outputs(d_cnt, nb, d_block_events, d_events, st);
    const hipError_t r = hipSetDevice(prev);
    if (e != hipSuccess)
        return fail(FSKMC_EDEVICE, "allocation-free advance: %s", hipGetErrorString(e));
    if (r != hipSuccess)
        return fail(FSKMC_EDEVICE, "hipSetDevice: %s", hipGetErrorString(r));
    return FSKMC_OK;
}

}  // extern "C"
