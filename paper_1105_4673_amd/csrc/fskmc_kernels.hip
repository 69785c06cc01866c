// HIP kernels of libfskmc for gfx950 (CDNA4, wave64).
//
// The sweep runs one fractional-step window (Sec. 2.2, the three-stage step;
// eqs. lie / strang with eq. exact): every block of the active colour runs a
// serial SSA kernel (Sec. 1, eqs. totalrate and skeleton) for the window's
// duration while all other sites stay frozen.  One wavefront owns one block:
//
//   * the block and its one-site halo are staged from HBM into a per-wave LDS
//     tile (coalesced row segments of P bytes per lane);
//   * leaf rates come from the host-built FP64 table (a per-wave LDS copy)
//     indexed by the site's neighbourhood;
//   * the canonical heap sum tree over the b*b leaves (row-major leaf order,
//     node = left + right) lives in VGPRs: each lane holds the pairwise tree
//     of its P consecutive leaves, and the top six levels are an xor
//     butterfly across the 64 lanes (a + b == b + a in IEEE, so every lane
//     holds exactly the node values of the heap tree);
//   * the descent is done by all lanes at once: lane j checks whether the
//     root-to-leaf path of its own subtree is the one the serial descent
//     takes, a ballot picks the single consistent lane, which finishes the
//     last log2(P) levels in registers;
//   * the Philox4x32-10 draws and their logarithms are computed 64 at a time,
//     one per lane, and broadcast with readlane as events consume them.
//
// All arithmetic on the decision path is FP64 with IEEE +,-,*,/ only and no
// contraction (built with -ffp-contract=off), so the results match the CPU
// statement of the scheme bit for bit.
#include "fskmc_internal.h"

#include <algorithm>

namespace fskmc {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the two
// multipliers 0xD2511F53, 0xCD9E8D57 with Weyl key increments 0x9E3779B9,
// 0xBB67AE85.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// U in (0,1] from words x,y and V in [0,1) from words z,w: top 53 bits.
__device__ __forceinline__ double unif_open0(uint4 r)
{
    const uint64_t a = ((uint64_t)r.x << 32) | r.y;
    return (double)((a >> 11) + 1u) * 0x1p-53;
}
__device__ __forceinline__ double unif_open1(uint4 r)
{
    const uint64_t b = ((uint64_t)r.z << 32) | r.w;
    return (double)(b >> 11) * 0x1p-53;
}

// Natural logarithm from IEEE +,-,*,/ and exact bit operations: u = m 2^e
// with m in [sqrt(1/2), sqrt(2)), s = (m-1)/(m+1), log m = 2s(1 + z/3 + ...
// + z^10/21) with z = s^2 (atanh series, Horner), plus e ln 2 split so that
// e * ln2_hi is exact.  Same steps, constants and operation order as the
// scheme's CPU statement; needs -ffp-contract=off.
__device__ __forceinline__ double fs_log(double u)
{
    long long bits = __double_as_longlong(u);
    int e = (int)((bits >> 52) & 0x7ff);
    if (e == 0) {
        u = u * 0x1p54;
        bits = __double_as_longlong(u);
        e = (int)((bits >> 52) & 0x7ff) - 54;
    }
    e -= 1023;
    double m = __longlong_as_double((bits & 0x000fffffffffffffLL) | 0x3ff0000000000000LL);
    if (m >= 0x1.6a09e667f3bcdp+0) {
        m = m * 0.5;
        e = e + 1;
    }
    const double f = m - 1.0;
    const double s = f / (2.0 + f);
    const double z = s * s;
    double P = 1.0 / 21.0;
    P = P * z + 1.0 / 19.0;
    P = P * z + 1.0 / 17.0;
    P = P * z + 1.0 / 15.0;
    P = P * z + 1.0 / 13.0;
    P = P * z + 1.0 / 11.0;
    P = P * z + 1.0 / 9.0;
    P = P * z + 1.0 / 7.0;
    P = P * z + 1.0 / 5.0;
    P = P * z + 1.0 / 3.0;
    const double two_s = s + s;
    const double logm = two_s + two_s * (z * P);
    const double ed = (double)e;
    return ed * 0x1.62e42ff000000p-1 + (ed * -0x1.718432a1b0e26p-35 + logm);
}

// ---------------------------------------------------------------------------
// Wave-level helpers.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __longlong_as_double(((long long)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double uniform_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const int hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __longlong_as_double(((long long)(uint32_t)hi << 32) | (uint32_t)lo);
}

// A lane's run of P consecutive sites of one block row, as packed bytes.
template <int P>
struct Seg {
    uint32_t w[(P + 3) / 4];
};

template <int P>
__device__ __forceinline__ uint32_t byte_at(const Seg<P>& s, int q)
{
    return (s.w[q >> 2] >> ((q & 3) * 8)) & 0xffu;
}

template <int P>
__device__ __forceinline__ Seg<P> load_seg(const uint8_t* p)
{
    Seg<P> s;
    if constexpr (P == 1) {
        s.w[0] = *p;
    } else if constexpr (P == 4) {
        s.w[0] = *reinterpret_cast<const uint32_t*>(p);
    } else {
        static_assert(P == 16, "P");
        const uint4 v = *reinterpret_cast<const uint4*>(p);
        s.w[0] = v.x;
        s.w[1] = v.y;
        s.w[2] = v.z;
        s.w[3] = v.w;
    }
    return s;
}

template <int P>
__device__ __forceinline__ void store_seg(uint8_t* p, const Seg<P>& s)
{
    if constexpr (P == 1) {
        *p = (uint8_t)s.w[0];
    } else if constexpr (P == 4) {
        *reinterpret_cast<uint32_t*>(p) = s.w[0];
    } else {
        *reinterpret_cast<uint4*>(p) = make_uint4(s.w[0], s.w[1], s.w[2], s.w[3]);
    }
}

// Compile-time geometry of one sweep variant.  BX x BY = 64 P sites; lane j
// owns leaves [jP, (j+1)P), i.e. row j / (BX/P), columns (j % (BX/P)) P + q.
template <int P, int BX, int BY, int MODEL>
struct Cfg {
    static_assert(BX * BY == 64 * P, "one wave per block");
    static_assert(BX % P == 0, "a lane's sites lie in one row");
    static constexpr int DIM = BY == 1 ? 1 : 2;
    static constexpr int Z = 2 * DIM;
    static constexpr int S = BX + 2 * P;                 // tile row stride
    static constexpr int TILE = ((BY + 2) * S + 15) / 16 * 16;
    static constexpr int NTAB = MODEL == MODEL_FLIP ? 2 * (Z + 1) : 243;
    static constexpr int LDS = TILE + NTAB * 8;          // bytes per wave
    static constexpr int LPR = BX / P;                   // lanes per row
    static constexpr int LOGP = P == 1 ? 0 : (P == 4 ? 2 : 4);
};

// Leaves of this lane from the LDS tile, then its in-lane pairwise tree and
// the cross-lane butterfly: g[s] = sum of the aligned group of 2^s lanes that
// contains this lane, pr[s] = that of the sibling group; g[6] = root.
template <int P, int BX, int BY, int MODEL>
__device__ __forceinline__ void build_tree(const uint8_t* tile, int tb, const double* tab, double (&lv)[2 * P],
                                           double (&g)[7], double (&pr)[6])
{
    using C = Cfg<P, BX, BY, MODEL>;
    const Seg<P> o = load_seg<P>(tile + tb);
    const uint32_t lft = tile[tb - 1], rgt = tile[tb + P];
    Seg<P> up, dn;
    if constexpr (C::DIM == 2) {
        up = load_seg<P>(tile + tb + C::S); // +y
        dn = load_seg<P>(tile + tb - C::S); // -y
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const uint32_t s = byte_at<P>(o, q);
        const uint32_t E = (q + 1 < P) ? byte_at<P>(o, q + 1) : rgt;
        const uint32_t W = (q > 0) ? byte_at<P>(o, q - 1) : lft;
        uint32_t N = 0, Sd = 0;
        if constexpr (C::DIM == 2) {
            N = byte_at<P>(up, q);
            Sd = byte_at<P>(dn, q);
        }
        uint32_t idx;
        if constexpr (MODEL == MODEL_FLIP)
            idx = s * (C::Z + 1) + E + W + N + Sd;
        else
            idx = s + 3 * E + 9 * W + 27 * N + 81 * Sd;
        lv[P + q] = tab[idx];
    }
#pragma unroll
    for (int k = P - 1; k >= 1; --k)
        lv[k] = lv[2 * k] + lv[2 * k + 1];
    g[0] = lv[1];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        pr[s] = __shfl_xor(g[s], 1 << s, 64);
        g[s + 1] = g[s] + pr[s];
    }
}

// One block-window.  `lds` is this wave's private LDS slice.
template <int P, int BX, int BY, int MODEL>
__device__ void block_window(const BlockWork& bw, uint8_t* lds)
{
    using C = Cfg<P, BX, BY, MODEL>;
    const int lane = threadIdx.x & 63;
    uint8_t* tile = lds;
    double* tab = reinterpret_cast<double*>(lds + C::TILE);

    // rate table into LDS (flip: site rates; reaction model: site totals)
    for (int i = lane; i < C::NTAB; i += 64)
        tab[i] = (MODEL == MODEL_FLIP) ? bw.table[i] : bw.table[i * 14 + 13];

    // stage the block and its halo
    const int bi = bw.m % bw.NBX, bj = bw.m / bw.NBX;
    const int x0 = bi * BX, y0 = bj * BY;
    const int r = lane / C::LPR, c0 = (lane % C::LPR) * P;
    const int gy = y0 + r, gx = x0 + c0;
    const size_t Lx = (size_t)bw.Lx;
    uint8_t* grow = bw.lat + (size_t)gy * Lx;
    const int tb = (r + 1) * C::S + P + c0;
    const bool has_top = C::DIM == 2 && r == 0;
    const bool has_bot = C::DIM == 2 && r == BY - 1;
    const bool has_l = c0 == 0, has_r = c0 + P == BX;
    const int xl = (x0 == 0 ? bw.Lx : x0) - 1;
    const int xr = (x0 + BX == bw.Lx) ? 0 : x0 + BX;
    uint8_t* gtop = bw.lat + (size_t)(gy == 0 ? bw.Ly - 1 : gy - 1) * Lx + gx;
    uint8_t* gbot = bw.lat + (size_t)(gy + 1 == bw.Ly ? 0 : gy + 1) * Lx + gx;
    {
        const Seg<P> own = load_seg<P>(grow + gx);
        Seg<P> top, bot;
        uint32_t lb = 0, rb = 0;
        if (has_top)
            top = load_seg<P>(gtop);
        if (has_bot)
            bot = load_seg<P>(gbot);
        if (has_l)
            lb = grow[xl];
        if (has_r)
            rb = grow[xr];
        store_seg<P>(tile + tb, own);
        if (has_top)
            store_seg<P>(tile + tb - C::S, top);
        if (has_bot)
            store_seg<P>(tile + tb + C::S, bot);
        if (has_l)
            tile[tb - 1] = (uint8_t)lb;
        if (has_r)
            tile[tb + P] = (uint8_t)rb;
    }
    wave_sync();

    double lv[2 * P], g[7], pr[6];
    build_tree<P, BX, BY, MODEL>(tile, tb, tab, lv, g, pr);

    double t = 0.0;
    uint32_t e = 0;
    uint32_t e0 = 0;
    double nl_b = 0.0, v_b = 0.0; // this lane's draw e0 + lane: -log U and V
    bool have_batch = false;
    for (;;) {
        const double R = uniform_f64(g[6]);
        if (R == 0.0)
            break;
        if (!have_batch || e - e0 >= 64u) {
            e0 = have_batch ? e : 0u;
            have_batch = true;
            const uint4 rr = philox10(make_uint4(e0 + (uint32_t)lane, (uint32_t)bw.m, bw.w, 0u), bw.k0, bw.k1);
            nl_b = -fs_log(unif_open0(rr));
            v_b = unif_open1(rr);
        }
        const int k = (int)(e - e0);
        const double nl = readlane_f64(nl_b, k);
        const double V = readlane_f64(v_b, k);
        const double tn = t + nl / R;
        if (!(tn < bw.dur))
            break;
        t = tn;

        // descent, top six levels: is this lane's subtree on the path?
        double tl = V * R;
        bool ok = true;
#pragma unroll
        for (int s = 5; s >= 0; --s) {
            const bool bit = (lane >> s) & 1;
            const double left = bit ? pr[s] : g[s];
            const double right = bit ? g[s] : pr[s];
            const bool go_right = !(tl < left || right == 0.0);
            ok = ok && (go_right == bit);
            if (go_right)
                tl = tl - left;
        }
        // the remaining log2(P) levels inside the lane
        int kk = 1;
#pragma unroll
        for (int lev = 0; lev < C::LOGP; ++lev) {
            const int width = 1 << lev;
            double L = lv[2 * width], Rr = lv[2 * width + 1];
#pragma unroll
            for (int c = 1; c < width; ++c) {
                if (kk - width == c) {
                    L = lv[2 * (width + c)];
                    Rr = lv[2 * (width + c) + 1];
                }
            }
            const bool go_right = !(tl < L || Rr == 0.0);
            if (go_right)
                tl = tl - L;
            kk = 2 * kk + (go_right ? 1 : 0);
        }
        const uint64_t bal = __ballot(ok);
        const int js = __ffsll((unsigned long long)bal) - 1;
        const int q = __builtin_amdgcn_readlane(kk - P, js);
        const int leaf = js * P + q;
        const int lx = leaf % BX, ly = leaf / BX;
        const int ts = (ly + 1) * C::S + P + lx;

        if constexpr (MODEL == MODEL_FLIP) {
            if (lane == 0)
                tile[ts] = (uint8_t)(tile[ts] ^ 1u);
        } else {
            double tg = readlane_f64(tl, js);
            const uint32_t s = tile[ts];
            const uint32_t nE = tile[ts + 1], nW = tile[ts - 1], nN = tile[ts + C::S], nS = tile[ts - C::S];
            const int pat = (int)(s + 3 * nE + 9 * nW + 27 * nN + 81 * nS);
            const double* ch = bw.table + pat * 14;
            int pick = -1, last = -1;
            for (int c = 0; c < 13; ++c) {
                const double rc = ch[c];
                if (rc == 0.0)
                    continue;
                last = c;
                if (tg < rc) {
                    pick = c;
                    break;
                }
                tg = tg - rc;
            }
            if (pick < 0)
                pick = last;
            if (lane == 0) {
                if (pick == 0) {
                    tile[ts] = 1;
                } else {
                    const int d = (pick - 1) & 3;
                    const int off = d == 0 ? 1 : d == 1 ? -1 : d == 2 ? C::S : -C::S;
                    if (pick <= 4) {
                        tile[ts] = 2;
                        tile[ts + off] = 2;
                    } else if (pick <= 8) {
                        tile[ts] = 0;
                        tile[ts + off] = 0;
                    } else {
                        tile[ts] = 0;
                        tile[ts + off] = 1;
                    }
                }
            }
        }
        wave_sync();
        build_tree<P, BX, BY, MODEL>(tile, tb, tab, lv, g, pr);
        ++e;
        if (e == 0xFFFFFFFFu)
            break; // the draw counter is 32-bit; a window never gets here in practice
    }

    // write back: the block (spin flip), the block and its halo (pair model)
    if (e > 0) {
        store_seg<P>(grow + gx, load_seg<P>(tile + tb));
        if constexpr (MODEL == MODEL_ZGB) {
            if (has_top)
                store_seg<P>(gtop, load_seg<P>(tile + tb - C::S));
            if (has_bot)
                store_seg<P>(gbot, load_seg<P>(tile + tb + C::S));
            if (has_l)
                grow[xl] = tile[tb - 1];
            if (has_r)
                grow[xr] = tile[tb + P];
        }
    }
    if (lane == 0) {
        bw.W_last[bw.m] = e;
        bw.cum_events[bw.m] += e;
        bw.cum_writes[bw.m] += (e > 0) ? 1u : 0u;
    }
}

template <int P, int BX, int BY, int MODEL, int WPG>
__global__ __launch_bounds__(64 * WPG) void k_sweep_single(SweepArgs a)
{
    using C = Cfg<P, BX, BY, MODEL>;
    __shared__ __attribute__((aligned(16))) uint8_t lds[WPG * C::LDS];
    const int wid = threadIdx.x >> 6;
    const int item = blockIdx.x * WPG + wid;
    if (item >= a.n_blocks)
        return; // the whole wave leaves; waves never synchronise with each other
    BlockWork bw;
    bw.lat = a.lat;
    bw.table = a.table;
    bw.W_last = a.W_last;
    bw.cum_events = a.cum_events;
    bw.cum_writes = a.cum_writes;
    bw.Lx = a.Lx;
    bw.Ly = a.Ly;
    bw.m = a.blocks[item];
    bw.NBX = a.NBX;
    bw.k0 = a.k0;
    bw.k1 = a.k1;
    bw.w = a.w;
    bw.dur = a.dur;
    block_window<P, BX, BY, MODEL>(bw, lds + wid * C::LDS);
}

template <int P, int BX, int BY, int MODEL, int WPG>
__global__ __launch_bounds__(64 * WPG) void k_sweep_batched(const JobDesc* __restrict__ jobs,
                                                            const uint32_t* __restrict__ item_job,
                                                            uint32_t n_items, uint64_t step)
{
    using C = Cfg<P, BX, BY, MODEL>;
    __shared__ __attribute__((aligned(16))) uint8_t lds[WPG * C::LDS];
    const int wid = threadIdx.x >> 6;
    const uint32_t item = blockIdx.x * WPG + wid;
    if (item >= n_items)
        return;
    const uint32_t j = item_job[item];
    const JobDesc& jd = jobs[j];
    const uint64_t w = jd.base_window + step;
    if (w >= jd.n_windows)
        return;
    const int c = jd.win_colour[w];
    const uint32_t k = item - jd.item_begin;
    const int beg = jd.colour_off[c], end = jd.colour_off[c + 1];
    if (k >= (uint32_t)(end - beg))
        return;
    BlockWork bw;
    bw.lat = jd.lat;
    bw.table = jd.table;
    bw.W_last = jd.W_last;
    bw.cum_events = jd.cum_events;
    bw.cum_writes = jd.cum_writes;
    bw.Lx = jd.Lx;
    bw.Ly = jd.Ly;
    bw.m = jd.blocks[beg + k];
    bw.NBX = jd.NBX;
    bw.k0 = jd.k0;
    bw.k1 = jd.k1;
    bw.w = (uint32_t)w;
    bw.dur = jd.win_dur[w];
    block_window<P, BX, BY, MODEL>(bw, lds + wid * C::LDS);
}

// ---------------------------------------------------------------------------
// Initial states and fills.
__global__ void k_init(uint8_t* lat, int64_t n, int kind, double p, uint32_t k0, uint32_t k1)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint8_t v = 0;
        if (kind == 1) {
            const uint4 r = philox10(make_uint4((uint32_t)i, 0u, 0u, 1u), k0, k1);
            v = unif_open1(r) < p ? 1 : 0;
        }
        lat[i] = v;
    }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Observables: per state k the number of sites and of nearest-neighbour bonds
// (+x and, in 2D, +y) with both ends k; the A-B bonds; and the sums of the
// per-block event and write-back counters.  Each thread takes four
// consecutive sites.
__global__ void k_observe(const uint8_t* __restrict__ lat, int Lx, int Ly, int dim,
                          const uint64_t* __restrict__ cum_events, const uint32_t* __restrict__ cum_writes,
                          int n_blocks, unsigned long long* out)
{
    unsigned long long acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t nq = (int64_t)Lx * Ly / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nq; i += stride) {
        const int64_t s0 = 4 * i;
        const int y = (int)(s0 / Lx), x = (int)(s0 % Lx);
        const uint32_t own = *reinterpret_cast<const uint32_t*>(lat + s0);
        const uint32_t nxt = lat[(int64_t)y * Lx + (x + 4 == Lx ? 0 : x + 4)];
        uint32_t up = 0;
        if (dim == 2)
            up = *reinterpret_cast<const uint32_t*>(lat + (int64_t)(y + 1 == Ly ? 0 : y + 1) * Lx + x);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t s = (own >> (8 * q)) & 0xffu;
            const uint32_t rx = q < 3 ? (own >> (8 * (q + 1))) & 0xffu : nxt;
            acc[s] += 1;
            acc[3 + s] += (rx == s);
            acc[6] += ((s == 1 && rx == 2) || (s == 2 && rx == 1));
            if (dim == 2) {
                const uint32_t ry = (up >> (8 * q)) & 0xffu;
                acc[3 + s] += (ry == s);
                acc[6] += ((s == 1 && ry == 2) || (s == 2 && ry == 1));
            }
        }
    }
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < n_blocks; b += stride) {
        acc[7] += cum_events[b];
        acc[8] += cum_writes[b];
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        unsigned long long v = acc[c];
        for (int o = 32; o >= 1; o >>= 1)
            v += __shfl_xor(v, o, 64);
        if ((threadIdx.x & 63) == 0 && v)
            atomicAdd(out + c, v);
    }
}

// ---------------------------------------------------------------------------
// Dispatch.
template <int MODEL, int WPG>
static hipError_t sweep_single_dispatch(int P, int shape, const SweepArgs& a, hipStream_t s)
{
    const dim3 grid((a.n_blocks + WPG - 1) / WPG), block(64 * WPG);
    if (shape == SHAPE_SQ) {
        if (P == 1)
            hipLaunchKernelGGL((k_sweep_single<1, 8, 8, MODEL, WPG>), grid, block, 0, s, a);
        else if (P == 4)
            hipLaunchKernelGGL((k_sweep_single<4, 16, 16, MODEL, WPG>), grid, block, 0, s, a);
        else if (P == 16)
            hipLaunchKernelGGL((k_sweep_single<16, 32, 32, MODEL, WPG>), grid, block, 0, s, a);
        else
            return hipErrorInvalidValue;
    } else {
        if constexpr (MODEL != MODEL_FLIP) {
            return hipErrorInvalidValue;
        } else {
            if (P == 1)
                hipLaunchKernelGGL((k_sweep_single<1, 64, 1, MODEL, WPG>), grid, block, 0, s, a);
            else if (P == 4)
                hipLaunchKernelGGL((k_sweep_single<4, 256, 1, MODEL, WPG>), grid, block, 0, s, a);
            else if (P == 16)
                hipLaunchKernelGGL((k_sweep_single<16, 1024, 1, MODEL, WPG>), grid, block, 0, s, a);
            else
                return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

template <int MODEL, int WPG>
static hipError_t sweep_batched_dispatch(int P, int shape, const JobDesc* jobs, const uint32_t* item_job,
                                         uint32_t n_items, uint64_t step, hipStream_t s)
{
    const dim3 grid((n_items + WPG - 1) / WPG), block(64 * WPG);
    if (shape == SHAPE_SQ) {
        if (P == 1)
            hipLaunchKernelGGL((k_sweep_batched<1, 8, 8, MODEL, WPG>), grid, block, 0, s, jobs, item_job, n_items, step);
        else if (P == 4)
            hipLaunchKernelGGL((k_sweep_batched<4, 16, 16, MODEL, WPG>), grid, block, 0, s, jobs, item_job, n_items, step);
        else if (P == 16)
            hipLaunchKernelGGL((k_sweep_batched<16, 32, 32, MODEL, WPG>), grid, block, 0, s, jobs, item_job, n_items, step);
        else
            return hipErrorInvalidValue;
    } else {
        if constexpr (MODEL != MODEL_FLIP) {
            return hipErrorInvalidValue;
        } else {
            if (P == 1)
                hipLaunchKernelGGL((k_sweep_batched<1, 64, 1, MODEL, WPG>), grid, block, 0, s, jobs, item_job, n_items, step);
            else if (P == 4)
                hipLaunchKernelGGL((k_sweep_batched<4, 256, 1, MODEL, WPG>), grid, block, 0, s, jobs, item_job, n_items, step);
            else if (P == 16)
                hipLaunchKernelGGL((k_sweep_batched<16, 1024, 1, MODEL, WPG>), grid, block, 0, s, jobs, item_job, n_items, step);
            else
                return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_sweep_single(int model, int P, int shape, int wpg, const SweepArgs& a, hipStream_t s)
{
    if (a.n_blocks <= 0)
        return hipSuccess;
#define FSKMC_SW(MOD)                                                          \
    switch (wpg) {                                                             \
    case 1: return sweep_single_dispatch<MOD, 1>(P, shape, a, s);              \
    case 2: return sweep_single_dispatch<MOD, 2>(P, shape, a, s);              \
    case 4: return sweep_single_dispatch<MOD, 4>(P, shape, a, s);              \
    case 8: return sweep_single_dispatch<MOD, 8>(P, shape, a, s);              \
    default: return hipErrorInvalidValue;                                      \
    }
    if (model == MODEL_FLIP) {
        FSKMC_SW(MODEL_FLIP)
    } else {
        FSKMC_SW(MODEL_ZGB)
    }
#undef FSKMC_SW
}

hipError_t launch_sweep_batched(int model, int P, int shape, int wpg, const JobDesc* jobs, const uint32_t* item_job,
                                uint32_t n_items, uint64_t step, hipStream_t s)
{
    if (n_items == 0)
        return hipSuccess;
#define FSKMC_SW(MOD)                                                                        \
    switch (wpg) {                                                                           \
    case 1: return sweep_batched_dispatch<MOD, 1>(P, shape, jobs, item_job, n_items, step, s); \
    case 2: return sweep_batched_dispatch<MOD, 2>(P, shape, jobs, item_job, n_items, step, s); \
    case 4: return sweep_batched_dispatch<MOD, 4>(P, shape, jobs, item_job, n_items, step, s); \
    case 8: return sweep_batched_dispatch<MOD, 8>(P, shape, jobs, item_job, n_items, step, s); \
    default: return hipErrorInvalidValue;                                                    \
    }
    if (model == MODEL_FLIP) {
        FSKMC_SW(MODEL_FLIP)
    } else {
        FSKMC_SW(MODEL_ZGB)
    }
#undef FSKMC_SW
}

static unsigned grid_for(int64_t n, int bs)
{
    int64_t g = (n + bs - 1) / bs;
    if (g < 1)
        g = 1;
    if (g > 65536)
        g = 65536;
    return (unsigned)g;
}

hipError_t launch_init(uint8_t* lat, int64_t n, int kind, double p, uint32_t k0, uint32_t k1, hipStream_t s)
{
    hipLaunchKernelGGL(k_init, dim3(grid_for(n, 256)), dim3(256), 0, s, lat, n, kind, p, k0, k1);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_observe(const uint8_t* lat, int Lx, int Ly, int dim, const uint64_t* cum_events,
                          const uint32_t* cum_writes, int n_blocks, unsigned long long* out9, hipStream_t s)
{
    const int64_t work = std::max<int64_t>((int64_t)Lx * Ly / 4, n_blocks);
    hipLaunchKernelGGL(k_observe, dim3(grid_for(work, 256) > 2048 ? 2048 : grid_for(work, 256)), dim3(256), 0, s,
                       lat, Lx, Ly, dim, cum_events, cum_writes, n_blocks, out9);
    return hipGetLastError();
}

}  // namespace fskmc
