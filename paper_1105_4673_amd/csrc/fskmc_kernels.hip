// HIP kernels of libfskmc for gfx950 (CDNA4, wave64).
//
// The sweep runs one fractional-step window (Sec. 2.2, the three-stage step;
// eqs. lie / strang with eq. exact): every block of the active colour runs a
// serial SSA kernel (Sec. 1, eqs. totalrate and skeleton) for the window's
// duration while all other sites stay frozen.  One wavefront owns one block:
//
//   * the block and its one-site halo are staged from HBM into a per-wave LDS
//     tile (row segments of P bytes per lane), with an XCD-aware block order
//     so that blocks sharing cache lines are served by the same L2;
//   * leaf rates come from the host-built FP64 table (a per-wave LDS copy)
//     indexed by the site's neighbourhood;
//   * the canonical heap sum tree over the leaves (row-major leaf order,
//     node = left + right) lives in registers: each lane holds the pairwise
//     tree of its P consecutive leaves; for the next four levels every lane
//     holds the left and right child sums of its group, fetched with DPP lane
//     moves inside each 16-lane row (quad_perm, and row shifts restricted to
//     the banks that need them), and the two top levels are the row and half
//     sums.  Since a + b == b + a in IEEE arithmetic, every lane holds
//     exactly the node values of the heap tree;
//   * the descent runs on all 64 lanes at once: each lane follows the path
//     of its own lane bits, applies the serial rule with its node's child
//     sums and stays in a 64-bit ballot mask while every decision agrees; the
//     last log2(P) levels run in registers, every lane on its own subtree,
//     and the single consistent lane's result is kept (with 16 sites per lane
//     in full launches that lane's leaves go to 16 lanes through LDS instead);
//   * the Philox4x32-10 draws and their logarithms are computed 64 at a time,
//     one per lane, and broadcast with readlane as events consume them.
//
// All arithmetic on the decision path is FP64 with IEEE +,-,*,/ only and no
// contraction (built with -ffp-contract=off), so the results match the CPU
// statement of the scheme bit for bit.
#include "fskmc_internal.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <utility>
#include <vector>

namespace fskmc {

// ---------------------------------------------------------------------------
// a ^ b ^ c in one instruction (v_bitop3_b32, truth table 0x96: set where an
// odd number of the three inputs is set); the compiler emits two XORs.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the two
// multipliers 0xD2511F53, 0xCD9E8D57 with Weyl key increments 0x9E3779B9,
// 0xBB67AE85.  Each round's two 32x32-bit products are taken whole (one
// v_mad_u64_u32 per product instead of separate low and high multiplies:
// 1.25x the generator's throughput, the same bits).
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4(xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1, xor3((uint32_t)(p0 >> 32), c.w, k1),
                       (uint32_t)p0);
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

// Value of a double in another lane through a DPP lane move that writes every
// lane (CTRL is the gfx9 DPP control, e.g. quad_perm 0x00-0xFF).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, true);
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

// Lattice accesses that are coherent across CUs and XCDs by themselves
// (relaxed agent-scope atomics: each load and store goes to the coherence
// point), used where other waves of the same kernel read what this wave
// wrote; no whole-cache write-back or invalidation is needed around them.
template <typename T>
__device__ __forceinline__ T coh_load(const T* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void coh_store(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int P, bool COH>
__device__ __forceinline__ Seg<P> gload_seg(const uint8_t* p)
{
    if constexpr (!COH) {
        return load_seg<P>(p);
    } else {
        Seg<P> s;
        if constexpr (P == 1) {
            s.w[0] = coh_load(p);
        } else {
#pragma unroll
            for (int k = 0; k < P / 4; ++k)
                s.w[k] = coh_load(reinterpret_cast<const uint32_t*>(p) + k);
        }
        return s;
    }
}

template <int P, bool COH>
__device__ __forceinline__ void gstore_seg(uint8_t* p, const Seg<P>& s)
{
    if constexpr (!COH) {
        store_seg<P>(p, s);
    } else {
        if constexpr (P == 1) {
            coh_store(p, (uint8_t)s.w[0]);
        } else {
#pragma unroll
            for (int k = 0; k < P / 4; ++k)
                coh_store(reinterpret_cast<uint32_t*>(p) + k, s.w[k]);
        }
    }
}

template <bool COH>
__device__ __forceinline__ uint32_t gload_byte(const uint8_t* p)
{
    if constexpr (COH)
        return coh_load(p);
    else
        return *p;
}

template <bool COH>
__device__ __forceinline__ void gstore_byte(uint8_t* p, uint32_t v)
{
    if constexpr (COH)
        coh_store(p, (uint8_t)v);
    else
        *p = (uint8_t)v;
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
    static constexpr int XFER = P == 16 ? 16 * 8 : 0;    // in-lane descent exchange
    static constexpr int LDS = TILE + NTAB * 8 + XFER;   // bytes per wave
    static constexpr int LPR = BX / P;                   // lanes per row
    static constexpr int LOGP = P == 1 ? 0 : (P == 4 ? 2 : 4);
};

// The block's sum tree.  Per lane: lv = pairwise tree of its P leaves
// (lv[1] lane sum, lv[P+q] leaf q).  Level s = 0..3 of a 16-lane row: L[s]
// and Rt[s] = the sums of the left and right halves of the aligned group of
// 2^(s+1) lanes that contains the lane; level 4: L4 / Rt4 = the two row sums
// of the lane's 32-lane half; level 5: h0 / h1 = the two half sums; R = root.
// Every value is the heap tree's node (node = left + right, which is the same
// IEEE result in either operand order).
template <int P>
struct Tree {
    double lv[2 * P];
    double L[4], Rt[4];
    double L4, Rt4, h0, h1, R;
};

// DPP lane move of a double: lanes enabled by BANK (4-lane banks of each
// 16-lane row) take the value from the lane CTRL selects, the others keep
// `old`.  CTRL (gfx9): quad_perm 0x00-0xFF, row_shl:n 0x100+n, row_shr:n
// 0x110+n.
template <int CTRL, int BANK>
__device__ __forceinline__ double dpp_keep_f64(double old, double v)
{
    const long long b = __double_as_longlong(v), o = __double_as_longlong(old);
    const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)b, CTRL, 0xF, BANK, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(b >> 32), CTRL, 0xF, BANK, false);
    return __longlong_as_double(((long long)(uint32_t)hi << 32) | (uint32_t)lo);
}

// The four levels of a 16-lane row from x (this lane's subtree sum): the left
// and right child sums of every lane's group at each level, fetched with DPP
// from the lane of the left (right) group, or kept where the lane is in that
// group.  Returns the row's sum.
__device__ __forceinline__ double row_tree(double x, double (&L)[4], double (&Rt)[4])
{
    L[0] = dpp_f64<0xA0>(x);  // quad_perm [0,0,2,2]
    Rt[0] = dpp_f64<0xF5>(x); // quad_perm [1,1,3,3]
    x = L[0] + Rt[0];
    L[1] = dpp_f64<0x44>(x);  // quad_perm [0,1,0,1]
    Rt[1] = dpp_f64<0xEE>(x); // quad_perm [2,3,2,3]
    x = L[1] + Rt[1];
    L[2] = dpp_keep_f64<0x114, 0xA>(x, x); // row_shr:4 into banks 1, 3
    Rt[2] = dpp_keep_f64<0x104, 0x5>(x, x); // row_shl:4 into banks 0, 2
    x = L[2] + Rt[2];
    L[3] = dpp_keep_f64<0x118, 0xC>(x, x); // row_shr:8 into banks 2, 3
    Rt[3] = dpp_keep_f64<0x108, 0x3>(x, x); // row_shl:8 into banks 0, 1
    return L[3] + Rt[3];
}

// Lanes whose bit S is set (the lanes whose path goes right at level S).
template <int S>
__device__ __forceinline__ constexpr uint64_t lanes_right()
{
    uint64_t m = 0;
    for (int l = 0; l < 64; ++l)
        if ((l >> S) & 1)
            m |= 1ull << l;
    return m;
}

// One level of the lane-parallel descent: every lane follows the path given
// by its own lane bits, with (left, right) the child sums of its node at this
// level.  The serial rule (go right iff not (tg < left or right == 0)) must
// agree with the lane's bit S for the lane to stay in `ok`.  The residual is
// fma(-left, bitf, tl) with bitf = 1.0 on paths that go right and 0.0 on the
// others: the product is exact, so this is tl - left rounded once, or tl.
template <int S>
__device__ __forceinline__ void path_level(double& tl, uint64_t& ok, int lane, double left, double right)
{
    const uint64_t not_below = __builtin_amdgcn_ballot_w64(!(tl < left));
    const uint64_t nonzero = __builtin_amdgcn_ballot_w64(right != 0.0);
    const uint64_t right_taken = not_below & nonzero;
    ok &= ~(right_taken ^ lanes_right<S>());
    tl = __builtin_fma(-left, ((lane >> S) & 1) ? 1.0 : 0.0, tl);
}

// Four descent levels inside a 16-lane row (row_tree's L, Rt).
__device__ __forceinline__ double row_descend(const double (&L)[4], const double (&Rt)[4], double tl, int lane,
                                              uint64_t& ok)
{
    path_level<3>(tl, ok, lane, L[3], Rt[3]);
    path_level<2>(tl, ok, lane, L[2], Rt[2]);
    path_level<1>(tl, ok, lane, L[1], Rt[1]);
    path_level<0>(tl, ok, lane, L[0], Rt[0]);
    return tl;
}

// Cross-row moves of a double with v_permlane16_swap / v_permlane32_swap
// (ROWS = 16 or 32), both operands the same value: `lo` receives the value of
// the lower row (half) of each pair in both, `hi` that of the upper.
constexpr bool kTopPermlane = true;

template <int ROWS>
__device__ __forceinline__ void swap_f64(double v, double& lo, double& hi)
{
    const long long b = __double_as_longlong(v);
    const unsigned l = (unsigned)(uint32_t)b, h = (unsigned)(uint32_t)(b >> 32);
    unsigned a0, a1, c0, c1;
    if constexpr (ROWS == 16) {
        const auto rl = __builtin_amdgcn_permlane16_swap(l, l, false, false);
        const auto rh = __builtin_amdgcn_permlane16_swap(h, h, false, false);
        a0 = rl[0]; a1 = rl[1]; c0 = rh[0]; c1 = rh[1];
    } else {
        const auto rl = __builtin_amdgcn_permlane32_swap(l, l, false, false);
        const auto rh = __builtin_amdgcn_permlane32_swap(h, h, false, false);
        a0 = rl[0]; a1 = rl[1]; c0 = rh[0]; c1 = rh[1];
    }
    lo = __longlong_as_double(((long long)c0 << 32) | a0);
    hi = __longlong_as_double(((long long)c1 << 32) | a1);
}

// In-lane pairwise levels, the row levels and the two top levels, from the
// leaves in T.lv[P..2P).
template <int P>
__device__ __forceinline__ void finish_tree(Tree<P>& T)
{
#pragma unroll
    for (int k = P - 1; k >= 1; --k)
        T.lv[k] = T.lv[2 * k] + T.lv[2 * k + 1];
    const double row = row_tree(T.lv[1], T.L, T.Rt);
    if constexpr (kTopPermlane) {
        // v_permlane16_swap with both operands = the row sums: the first
        // result holds the even row of each row pair in both rows, the second
        // the odd row; v_permlane32_swap does the same for the two halves
        swap_f64<16>(row, T.L4, T.Rt4);
        const double half = T.L4 + T.Rt4;
        swap_f64<32>(half, T.h0, T.h1);
    } else {
        double q4[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            q4[k] = readlane_f64(row, 16 * k);
        T.h0 = q4[0] + q4[1];
        T.h1 = q4[2] + q4[3];
        const bool upper = (threadIdx.x & 32) != 0;
        T.L4 = upper ? q4[2] : q4[0];
        T.Rt4 = upper ? q4[3] : q4[1];
    }
    T.R = T.h0 + T.h1;
}

// Leaves from the LDS tile: the table entry of each site's neighbourhood
// (spin flip: s*(z+1) + #occupied neighbours; reaction model: the pattern
// s + 3E + 9W + 27N + 81S).
// qmask (wave-uniform): bit q set = recompute leaf q of every lane; the
// other leaves keep their values.  The inner sums are always rebuilt, in the
// same order, so the tree equals a full rebuild whenever the skipped leaves
// are unchanged.
template <int P, int BX, int BY, int MODEL, int TS = BX + 2 * P>
__device__ __forceinline__ void build_tree(const uint8_t* tile, int tb, const double* tab, Tree<P>& T,
                                           uint32_t qmask = ~0u)
{
    using C = Cfg<P, BX, BY, MODEL>;
    const Seg<P> o = load_seg<P>(tile + tb);
    const uint32_t lft = tile[tb - 1], rgt = tile[tb + P];
    Seg<P> up, dn;
    if constexpr (C::DIM == 2) {
        up = load_seg<P>(tile + tb + TS); // +y
        dn = load_seg<P>(tile + tb - TS); // -y
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
        if (!((qmask >> q) & 1u))
            continue;
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
        T.lv[P + q] = tab[idx];
    }
    finish_tree(T);
}

// Spin flip: a lane's site states and occupied-neighbour counts as packed
// bytes, kept in registers for the whole window (the halo is frozen, so only
// flips inside the block change them).
template <int P>
struct FlipSites {
    uint32_t s[(P + 3) / 4], n[(P + 3) / 4];
};

// A lane's segment, the segments above and below it and the sites left and
// right of it: everything its sites' neighbour counts depend on.
template <int P>
struct FlipRows {
    Seg<P> o, up, dn;
    uint32_t lft, rgt;
};

template <int P, int BY, int S>
__device__ __forceinline__ FlipRows<P> flip_rows_from_tile(const uint8_t* tile, int tb)
{
    FlipRows<P> g;
    g.o = load_seg<P>(tile + tb);
    g.lft = tile[tb - 1];
    g.rgt = tile[tb + P];
    if constexpr (BY > 1) {
        g.up = load_seg<P>(tile + tb + S);
        g.dn = load_seg<P>(tile + tb - S);
    }
    return g;
}

template <int P, int BY>
__device__ __forceinline__ void flip_sites_from_rows(const FlipRows<P>& g, FlipSites<P>& F)
{
    constexpr int W = (P + 3) / 4;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        uint32_t Lw, Rw; // bytes of the -x and +x neighbours of each site
        if constexpr (P == 1) {
            Lw = g.lft;
            Rw = g.rgt;
        } else {
            Lw = (g.o.w[k] << 8) | (k > 0 ? g.o.w[k - 1] >> 24 : g.lft);
            Rw = (g.o.w[k] >> 8) | ((k + 1 < W ? (g.o.w[k + 1] & 0xffu) : g.rgt) << 24);
        }
        uint32_t n = Lw + Rw;
        if constexpr (BY > 1)
            n += g.up.w[k] + g.dn.w[k];
        F.s[k] = g.o.w[k];
        F.n[k] = n; // each byte <= 4: no carries between bytes
    }
}

template <int P, int BX, int BY, int S = BX + 2 * P>
__device__ __forceinline__ void flip_sites_from_tile(const uint8_t* tile, int tb, FlipSites<P>& F)
{
    flip_sites_from_rows<P, BY>(flip_rows_from_tile<P, BY, S>(tile, tb), F);
}

// Flip of block site (xi, yi) (uniform) to state v: toggle it and add +-1 to
// the counts of its in-block neighbours.  Site g of the block lives in lane
// g / P, byte g % P (row-major, P consecutive sites per lane).  Each lane
// finds its own bytes from the bit offset o = 8 (g - lane P) of site g from
// its first site: the site is held here iff 0 <= o < 8P, in word o >> 5 at
// bit o & 31.  Per site that is a few vector operations on the lane's own
// offset, instead of a scalar division and compare chain per site and word.
template <int P, int W>
__device__ __forceinline__ void site_bits(int o, uint32_t (&m)[W])
{
    const bool in = (uint32_t)o < (uint32_t)(8 * P);
    const uint32_t bit = 1u << (o & 31);
#pragma unroll
    for (int k = 0; k < W; ++k)
        m[k] |= (in && (W == 1 || (o >> 5) == k)) ? bit : 0u;
}

template <int P, int BX, int BY>
__device__ __forceinline__ void flip_apply(FlipSites<P>& F, int lane, int xi, int yi, bool v)
{
    constexpr int W = (P + 3) / 4;
    constexpr int FAR = 1 << 24; // moves a neighbour outside the block out of every lane's range
    const int o = 8 * (yi * BX + xi) - 8 * P * lane;
    const int dl = xi > 0 ? -8 : FAR;
    const int dr = xi < BX - 1 ? 8 : FAR;
    const int du = (BY > 1 && yi > 0) ? -8 * BX : FAR;
    const int dd = (BY > 1 && yi < BY - 1) ? 8 * BX : FAR;
    uint32_t own[W], nm[W];
#pragma unroll
    for (int k = 0; k < W; ++k)
        own[k] = nm[k] = 0u;
    site_bits<P, W>(o, own);
    site_bits<P, W>(o + dl, nm);
    site_bits<P, W>(o + dr, nm);
    site_bits<P, W>(o + du, nm);
    site_bits<P, W>(o + dd, nm);
    // counts + nm, or - nm as + (~nm + 1); no byte carries or borrows: a
    // count stays within 0..4
    const uint32_t flip = v ? 0u : ~0u, one = v ? 0u : 1u;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        F.s[k] ^= own[k];
        F.n[k] = F.n[k] + (nm[k] ^ flip) + one;
    }
}

template <int P, int Z>
__device__ __forceinline__ void flip_leaves(const FlipSites<P>& F, const double* tab, Tree<P>& T)
{
    // table index s (z+1) + n of four sites at once (bytes <= 2z+1: no carries)
    uint32_t idx[(P + 3) / 4];
#pragma unroll
    for (int k = 0; k < (P + 3) / 4; ++k)
        idx[k] = F.s[k] * (uint32_t)(Z + 1) + F.n[k];
#pragma unroll
    for (int q = 0; q < P; ++q)
        T.lv[P + q] = tab[(idx[q >> 2] >> (8 * (q & 3))) & 0xffu];
    finish_tree(T);
}

// Launches of at most this many blocks (two waves per SIMD) take the
// latency-bound variant of the 16-sites-per-lane descent (its own kernels).
constexpr int kLanePathBlocks = 2048;

// Descent of the heap tree with target tg in [0, R): at each node go left
// when tg < left or the right subtree is empty, else subtract left and go
// right.  Returns the leaf index within the block; *tg_out = residual target.
// P == 16 has two ways through the last four levels, the same path and bits:
// lane_path (every lane descends its own in-lane subtree, no memory; shorter
// latency, more instructions: for launches with few waves per SIMD) or
// through xfer, 16 doubles of this wave's LDS (for full launches).
template <int P>
__device__ __forceinline__ int descend(const Tree<P>& T, double tg, int lane, double* tg_out, double* xfer,
                                       bool lane_path)
{
    // six levels down to the lane, every lane on its own path
    uint64_t ok = ~0ull;
    double tl = tg;
    path_level<5>(tl, ok, lane, T.h0, T.h1);
    path_level<4>(tl, ok, lane, T.L4, T.Rt4);
    tl = row_descend(T.L, T.Rt, tl, lane, ok);
    int q = 0;
    if constexpr (P == 4) {
        // two levels inside the lane, in registers (constant indices only)
        bool gr = !(tl < T.lv[2] || T.lv[3] == 0.0);
        if (gr)
            tl = tl - T.lv[2];
        const double L = gr ? T.lv[6] : T.lv[4];
        const double Rr = gr ? T.lv[7] : T.lv[5];
        const bool gr2 = !(tl < L || Rr == 0.0);
        if (gr2)
            tl = tl - L;
        q = 2 * (gr ? 1 : 0) + (gr2 ? 1 : 0);
    }
    const int js = (__ffsll((unsigned long long)ok) - 1) & 63;
    if constexpr (P == 16) {
        if (!lane_path) {
            // lane js's 16 leaves go to lanes 0..15 through LDS, which rebuild
            // the four in-lane levels with the same row butterfly and descend:
            // fewer instructions, two LDS round trips
            const double tu = readlane_f64(tl, js);
            if (lane == js) {
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    xfer[i] = T.lv[16 + i];
            }
            wave_sync();
            double L2[4], R2[4];
            row_tree(xfer[lane & 15], L2, R2);
            uint64_t ok2 = 0xFFFFull; // lanes 0..15 hold the 16 leaves
            const double t2 = row_descend(L2, R2, tu, lane, ok2);
            q = (__ffsll((unsigned long long)ok2) - 1) & 15;
            *tg_out = readlane_f64(t2, q);
            wave_sync();
            return js * P + q;
        }
        // four levels inside every lane, on the lane's own residual (only lane
        // js's result is used), down its in-lane subtree: node k has children
        // 2k and 2k+1, leaves 16..31.  Nodes 2..7 come from the tree; the two
        // children of the level-3 node are the sums of its four leaves, added
        // as the tree adds them, and level 4 reads those leaves.  Children are
        // chosen with selects on the path bits, so registers are never indexed.
        const bool g1 = !(tl < T.lv[2] || T.lv[3] == 0.0);
        if (g1)
            tl = tl - T.lv[2];
        const double L2 = g1 ? T.lv[6] : T.lv[4];
        const double R2 = g1 ? T.lv[7] : T.lv[5];
        const bool g2 = !(tl < L2 || R2 == 0.0);
        if (g2)
            tl = tl - L2;
        double f[4]; // leaves 16 + 8 g1 + 4 g2 + i
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double lo = g1 ? T.lv[24 + i] : T.lv[16 + i];
            const double hi = g1 ? T.lv[28 + i] : T.lv[20 + i];
            f[i] = g2 ? hi : lo;
        }
        const double L3 = f[0] + f[1];
        const double R3 = f[2] + f[3];
        const bool g3 = !(tl < L3 || R3 == 0.0);
        if (g3)
            tl = tl - L3;
        const double L4 = g3 ? f[2] : f[0];
        const double R4 = g3 ? f[3] : f[1];
        const bool g4 = !(tl < L4 || R4 == 0.0);
        if (g4)
            tl = tl - L4;
        q = 8 * (g1 ? 1 : 0) + 4 * (g2 ? 1 : 0) + 2 * (g3 ? 1 : 0) + (g4 ? 1 : 0);
        q = __builtin_amdgcn_readlane(q, js) & (P - 1);
        *tg_out = readlane_f64(tl, js);
        return js * P + q;
    } else {
        q = __builtin_amdgcn_readlane(q, js) & (P - 1);
        *tg_out = readlane_f64(tl, js);
        return js * P + q;
    }
}

// Draws e0 .. e0+63 of block m in window w, one per lane: (-log U, V).  Not
// inlined: the event loop then keeps none of the generator's and the
// logarithm's constants live (they pushed the kernel arguments out of the
// scalar registers into spill lanes, reloaded every window).
__device__ __noinline__ double2 draw_batch(uint32_t e0, uint32_t m, uint32_t w, uint32_t k0, uint32_t k1)
{
    const uint4 rr = philox10(make_uint4(e0 + (uint32_t)(threadIdx.x & 63), m, w, 0u), k0, k1);
    return make_double2(-fs_log(unif_open0(rr)), unif_open1(rr));
}

// The serial SSA kernel of one block for one window (Sec. 1, eqs. totalrate
// and skeleton) on the block's LDS tile.  Draw e uses Philox counter
// (e, m, w, 0); the draw whose time passes the window end is discarded.
// Spin flip keeps the block in registers during the window and puts it back
// into the tile at the end; pair events update the tile in place.
// Returns the number of accepted events.  With `pre`, (nl0, v0) are this
// lane's -log U and V of draw e = lane, computed by the caller ahead of time.
// With `fin` (spin flip), the lane's site states and neighbour counts come
// from the caller instead of the tile's block and halo.  lane_path: the
// descent's variant for 16 sites per lane (see descend).  With `fout` (spin
// flip), the lane's final segment is also returned in registers and the tile
// store is left to the caller's next wave sync.
// TS: row stride of the tile (the block's own tile by default; a larger
// shared tile when several waves hold the sub-blocks of one coarse cell, in
// which case `tile` points at the sub-block's origin minus one row and P columns).
template <int P, int BX, int BY, int MODEL, int TS = BX + 2 * P>
__device__ __forceinline__ uint32_t ssa_window(uint8_t* tile, double* tab, const double* __restrict__ chan, uint32_t m,
                                               uint32_t w, double dur, uint32_t k0, uint32_t k1, bool pre = false,
                                               double nl0 = 0.0, double v0 = 0.0, const FlipSites<P>* fin = nullptr,
                                               bool lane_path = true, Seg<P>* fout = nullptr)
{
    using C = Cfg<P, BX, BY, MODEL>;
    const int lane = threadIdx.x & 63;
    const int r = lane / C::LPR, c0 = (lane % C::LPR) * P;
    const int tb = (r + 1) * TS + P + c0;
    Tree<P> T;
    FlipSites<P> F;
    if constexpr (MODEL == MODEL_FLIP) {
        if (fin)
            F = *fin;
        else
            flip_sites_from_tile<P, BX, BY, TS>(tile, tb, F);
        flip_leaves<P, C::Z>(F, tab, T);
    } else {
        build_tree<P, BX, BY, MODEL, TS>(tile, tb, tab, T);
    }

    double t = 0.0;
    uint32_t e = 0, e0 = 0;
    double nl_b = nl0, v_b = v0; // this lane's draw e0 + lane: -log U and V
    if (!pre && uniform_f64(T.R) != 0.0) {
        const uint4 rr = philox10(make_uint4((uint32_t)lane, m, w, 0u), k0, k1);
        nl_b = -fs_log(unif_open0(rr));
        v_b = unif_open1(rr);
    }
    // draws e0 .. e0 + avail - 1 are in hand; the draw counter is 32-bit, so
    // the last batch stops at e = 2^32 - 1, where the window ends
    uint32_t avail = 64u;
    for (;;) {
        const double R = uniform_f64(T.R);
        if (e - e0 >= avail) { // rare: a window with more than 64 events
            if (e == 0xFFFFFFFFu)
                break;
            e0 = e;
            avail = 0xFFFFFFFFu - e < 64u ? 0xFFFFFFFFu - e : 64u;
            const double2 d = draw_batch(e0, m, w, k0, k1);
            nl_b = d.x;
            v_b = d.y;
        }
        const int k = (int)(e - e0);
        const double nl = readlane_f64(nl_b, k);
        const double V = readlane_f64(v_b, k);
        // R == 0 (no site can change) gives tn = +inf, or NaN when nl == 0:
        // either way the window ends here without an event
        const double tn = t + nl / R;
        if (!(tn < dur))
            break;
        t = tn;
        double tg;
        const int leaf = descend<P>(T, V * R, lane, &tg, tab + C::NTAB, lane_path);
        const int lx = leaf % BX, ly = leaf / BX;
        if constexpr (MODEL == MODEL_FLIP) {
            const int js = leaf / P, q = leaf % P;
            uint32_t word = 0;
#pragma unroll
            for (int kw = 0; kw < (P + 3) / 4; ++kw) {
                const uint32_t wv = (uint32_t)__builtin_amdgcn_readlane((int)F.s[kw], js);
                word = (q >> 2) == kw ? wv : word;
            }
            const bool was = (word >> (8 * (q & 3))) & 1u;
            flip_apply<P, BX, BY>(F, lane, lx, ly, !was);
            flip_leaves<P, C::Z>(F, tab, T);
        } else {
            const int ts = (ly + 1) * TS + P + lx;
            const uint32_t s = tile[ts];
            const uint32_t nE = tile[ts + 1], nW = tile[ts - 1], nN = tile[ts + TS], nS = tile[ts - TS];
            const int pat = __builtin_amdgcn_readfirstlane((int)(s + 3 * nE + 9 * nW + 27 * nN + 81 * nS));
            // the pattern's 13 channel rates through the scalar cache, all
            // issued before the first is used: the row address is the same in
            // every lane, so it is made uniform and read in the constant
            // address space (the table is read-only while kernels run); then
            // the serial pick: the first non-zero channel with the residual
            // below its rate, the residual reduced by each channel passed
            const uint64_t ca = (uint64_t)(uintptr_t)(chan + pat * 14);
            const uint64_t cu = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(ca >> 32)) << 32) |
                                (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)ca);
            const __attribute__((address_space(4))) double* cp =
                (const __attribute__((address_space(4))) double*)(uintptr_t)cu;
            double rc[13];
#pragma unroll
            for (int c = 0; c < 13; ++c)
                rc[c] = cp[c];
            int pick = -1, last = -1;
#pragma unroll
            for (int c = 0; c < 13; ++c) {
                if (rc[c] == 0.0)
                    continue;
                last = c;
                if (tg < rc[c]) {
                    pick = c;
                    break;
                }
                tg = tg - rc[c];
            }
            if (pick < 0)
                pick = last;
            if (lane == 0) {
                if (pick == 0) {
                    tile[ts] = 1;
                } else {
                    const int d = (pick - 1) & 3;
                    const int off = d == 0 ? 1 : d == 1 ? -1 : d == 2 ? TS : -TS;
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
            wave_sync();
            // only leaves whose neighbourhood holds a changed site can change:
            // the columns around the event site and its partner; a lane holds
            // columns c0 .. c0+P-1 with c0 a multiple of P, so these are the
            // leaves q = column mod P of every lane.  With 4 or fewer leaves
            // per lane those columns cover them all (a horizontal pair spans 4),
            // and looking every leaf up without the per-leaf branches lets the
            // lookups overlap.
            uint32_t qmask = ~0u;
            if constexpr (P > 4) {
                int xa = lx, xb = lx;
                if (pick > 0) {
                    const int d = (pick - 1) & 3;
                    xa = d == 1 ? lx - 1 : lx;
                    xb = d == 0 ? lx + 1 : lx;
                }
                xa = xa > 0 ? xa - 1 : 0;
                xb = xb < BX - 1 ? xb + 1 : BX - 1;
                qmask = 0;
                for (int x = xa; x <= xb; ++x)
                    qmask |= 1u << (x % P);
            }
            build_tree<P, BX, BY, MODEL, TS>(tile, tb, tab, T, qmask);
        }
        ++e;
    }
    if constexpr (MODEL == MODEL_FLIP) {
        Seg<P> o;
#pragma unroll
        for (int k = 0; k < (P + 3) / 4; ++k)
            o.w[k] = F.s[k];
        if (e > 0) {
            store_seg<P>(tile + tb, o);
            if (!fout)
                wave_sync();
        }
        if (fout)
            *fout = o;
    }
    return e;
}

// One block-window of the streaming sweep: stage block + halo from the
// lattice into LDS, run the SSA window, write back what may have changed
// (the block for spin flip; block and halo for pair events), update counters.
// COH: lattice accesses coherent across the device (persistent sweep).
template <int P, int BX, int BY, int MODEL, bool COH = false>
__device__ __forceinline__ void block_window(uint8_t* __restrict__ lat, const double* __restrict__ table, BlockCount* cnt, int Lx,
                             int Ly, int m, int NBX, uint32_t k0, uint32_t k1, uint32_t w, double dur, uint8_t* lds,
                             bool lane_path)
{
    using C = Cfg<P, BX, BY, MODEL>;
    const int lane = threadIdx.x & 63;
    uint8_t* tile = lds;
    double* tab = reinterpret_cast<double*>(lds + C::TILE);

    for (int i = lane; i < C::NTAB; i += 64)
        tab[i] = (MODEL == MODEL_FLIP) ? table[i] : table[i * 14 + 13];

    const int bi = m % NBX, bj = m / NBX;
    const int x0 = bi * BX, y0 = bj * BY;
    const int r = lane / C::LPR, c0 = (lane % C::LPR) * P;
    const int gy = y0 + r, gx = x0 + c0;
    const size_t sLx = (size_t)Lx;
    uint8_t* grow = lat + (size_t)gy * sLx;
    const int tb = (r + 1) * C::S + P + c0;
    const bool has_top = C::DIM == 2 && r == 0;
    const bool has_bot = C::DIM == 2 && r == BY - 1;
    const bool has_l = c0 == 0, has_r = c0 + P == BX;
    const int xl = (x0 == 0 ? Lx : x0) - 1;
    const int xr = (x0 + BX == Lx) ? 0 : x0 + BX;
    uint8_t* gtop = lat + (size_t)(gy == 0 ? Ly - 1 : gy - 1) * sLx + gx;
    uint8_t* gbot = lat + (size_t)(gy + 1 == Ly ? 0 : gy + 1) * sLx + gx;
    {
        const Seg<P> own = gload_seg<P, COH>(grow + gx);
        Seg<P> top, bot;
        uint32_t lb = 0, rb = 0;
        if (has_top)
            top = gload_seg<P, COH>(gtop);
        if (has_bot)
            bot = gload_seg<P, COH>(gbot);
        if (has_l)
            lb = gload_byte<COH>(grow + xl);
        if (has_r)
            rb = gload_byte<COH>(grow + xr);
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

    const uint32_t e = ssa_window<P, BX, BY, MODEL>(tile, tab, table, (uint32_t)m, w, dur, k0, k1, false, 0.0, 0.0,
                                                    nullptr, lane_path);

    if (e > 0) {
        gstore_seg<P, COH>(grow + gx, load_seg<P>(tile + tb));
        if constexpr (MODEL == MODEL_ZGB) {
            if (has_top)
                gstore_seg<P, COH>(gtop, load_seg<P>(tile + tb - C::S));
            if (has_bot)
                gstore_seg<P, COH>(gbot, load_seg<P>(tile + tb + C::S));
            if (has_l)
                gstore_byte<COH>(grow + xl, tile[tb - 1]);
            if (has_r)
                gstore_byte<COH>(grow + xr, tile[tb + P]);
        }
    }
    if (lane == 0) {
        cnt[m].W = e;
        if (e > 0) {
            atomicAdd(&cnt[m].writes, 1u);
            atomicAdd(&cnt[m].events, (unsigned long long)e);
        }
    }
}

// Workgroups are dispatched round-robin over the eight XCDs (L2 domains);
// give each XCD a contiguous range of work so neighbouring blocks, which
// share cache lines, are fetched by one L2.
__device__ __forceinline__ uint32_t xcd_order(uint32_t wg, uint32_t G)
{
    return (G & 7u) ? wg : (wg & 7u) * (G >> 3) + (wg >> 3);
}

// LANE: the descent's latency-bound variant for 16 sites per lane, compiled as
// its own kernel (k_sweep_single_lane) so the full-launch kernel keeps its
// register count and occupancy.
template <int P, int BX, int BY, int MODEL, int WPG, bool LANE>
__device__ __forceinline__ void sweep_single_body(const SweepArgs& a, uint8_t* lds)
{
    using C = Cfg<P, BX, BY, MODEL>;
    const int wid = threadIdx.x >> 6;
    const int item = (int)xcd_order(blockIdx.x, gridDim.x) * WPG + wid;
    if (item >= a.n_blocks)
        return; // the whole wave leaves; waves never synchronise with each other
    block_window<P, BX, BY, MODEL>(a.lat, a.table, a.cnt, a.Lx, a.Ly, a.blocks[item], a.NBX, a.k0, a.k1, a.w,
                                   a.dur, lds + wid * C::LDS, LANE);
}

template <int P, int BX, int BY, int MODEL, int WPG>
__global__ __launch_bounds__(64 * WPG) void k_sweep_single(SweepArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[WPG * Cfg<P, BX, BY, MODEL>::LDS];
    sweep_single_body<P, BX, BY, MODEL, WPG, false>(a, lds);
}

template <int P, int BX, int BY, int MODEL, int WPG>
__global__ __launch_bounds__(64 * WPG) void k_sweep_single_lane(SweepArgs a)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[WPG * Cfg<P, BX, BY, MODEL>::LDS];
    sweep_single_body<P, BX, BY, MODEL, WPG, true>(a, lds);
}

template <int P, int BX, int BY, int MODEL, int WPG, bool LANE>
__device__ __forceinline__ void sweep_batched_body(const JobDesc* __restrict__ jobs,
                                                   const uint32_t* __restrict__ item_job, uint32_t n_items,
                                                   uint64_t step, uint8_t* lds)
{
    using C = Cfg<P, BX, BY, MODEL>;
    const int wid = threadIdx.x >> 6;
    const uint32_t item = xcd_order(blockIdx.x, gridDim.x) * WPG + wid;
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
    block_window<P, BX, BY, MODEL>(jd.lat, jd.table, jd.cnt, jd.Lx, jd.Ly, jd.blocks[beg + k], jd.NBX, jd.k0,
                                   jd.k1, (uint32_t)w, jd.win_dur[w], lds + wid * C::LDS, LANE);
}

template <int P, int BX, int BY, int MODEL, int WPG>
__global__ __launch_bounds__(64 * WPG) void k_sweep_batched(const JobDesc* __restrict__ jobs,
                                                            const uint32_t* __restrict__ item_job,
                                                            uint32_t n_items, uint64_t step)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[WPG * Cfg<P, BX, BY, MODEL>::LDS];
    sweep_batched_body<P, BX, BY, MODEL, WPG, false>(jobs, item_job, n_items, step, lds);
}

// The batched sweep with the descent's latency-bound variant (16 sites per
// lane, small launches).
template <int P, int BX, int BY, int MODEL, int WPG>
__global__ __launch_bounds__(64 * WPG) void k_sweep_batched_lane(const JobDesc* __restrict__ jobs,
                                                                 const uint32_t* __restrict__ item_job,
                                                                 uint32_t n_items, uint64_t step)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[WPG * Cfg<P, BX, BY, MODEL>::LDS];
    sweep_batched_body<P, BX, BY, MODEL, WPG, true>(jobs, item_job, n_items, step, lds);
}

// Lanes 0..7 wait until each block that can interact with block m has
// finished its windows before w (epoch >= w), bounded by wait_ticks of the
// 100 MHz wall clock (then the abort flag is raised).  With `own`, lane 8
// also waits for block m's own earlier windows: needed when windows of one
// block may be taken by different waves, since two consecutive windows of
// one colour have no neighbour window between them.  True when the launch is
// aborting: every wave then leaves.
__device__ __forceinline__ bool wait_neighbours(const int32_t* nbr, const int32_t* epoch, int m, int w, int lane,
                                                int32_t* abort_flag, unsigned long long wait_ticks, bool own = false)
{
    if (lane < 8 || (own && lane == 8)) {
        const int nb = lane == 8 ? m : nbr[m * 8 + lane];
        if (nb >= 0) {
            const uint64_t t0 = wall_clock64();
            while (__hip_atomic_load(&epoch[nb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < w) {
                if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    break;
                if (wall_clock64() - t0 > wait_ticks) {
                    __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
    }
    return __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// Persistent multi-window sweep of one simulation (cooperative launch: every
// wave is resident).  Windows [w0, w1) run in order inside the kernel and the
// colour barrier becomes a neighbour-only wait, the local synchronisation of
// Sec. 2.2 stage 2: before block m runs window w, each block that can
// interact with it must have finished all its windows before w.  epoch[n] is
// the next window block n takes part in.  The lattice and the epochs are only
// touched with agent-coherent loads and stores (no whole-cache write-back or
// invalidation); an epoch is stored after the block's lattice stores have
// completed and lattice loads are issued after the epoch loads.  Same-colour
// blocks of one window never interact, windows only depend on earlier ones,
// so every wait ends; a wait longer than wait_ticks (100 MHz wall clock)
// raises the abort flag and every wave leaves.
template <int P, int BX, int BY, int MODEL, int WPG>
__global__ __launch_bounds__(64 * WPG) void k_sweep_persistent(PersistArgs a)
{
    using C = Cfg<P, BX, BY, MODEL>;
    __shared__ __attribute__((aligned(16))) uint8_t lds[WPG * C::LDS];
    const int wid = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int gw = (int)xcd_order(blockIdx.x, gridDim.x) * WPG + wid;
    for (int w = a.w0; w < a.w1; ++w) {
        const int c = a.win_colour[w];
        const int beg = a.colour_off[c], count = a.colour_off[c + 1] - beg;
        const int nxt = a.next_part[c * (a.n_windows + 1) + w + 1];
        for (int k = gw; k < count; k += a.n_waves) {
            const int m = a.blocks[beg + k];
            if (wait_neighbours(a.nbr, a.epoch, m, w, lane, a.abort_flag, a.wait_ticks))
                return;
            // issue priority over waves that are still waiting, until the
            // epoch that releases this block's neighbours is out
            __builtin_amdgcn_s_setprio(3);
            // the lattice is read and written with agent-coherent accesses, so
            // only their order matters here: loads after the epoch loads,
            // epoch store after the lattice stores have completed
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            block_window<P, BX, BY, MODEL, true>(a.lat, a.table, a.cnt, a.Lx, a.Ly, m, a.NBX, a.k0, a.k1,
                                                 (uint32_t)w, a.win_dur[w], lds + wid * C::LDS, true);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            // a workgroup-scope release does not wait for stores to complete;
            // the epoch must not be published before the block's agent-scope
            // lattice stores have been performed (vmcnt(0), other counters
            // left at their maxima)
            __builtin_amdgcn_s_waitcnt(0x0F70);
            if (lane == 0)
                __hip_atomic_store(&a.epoch[m], nxt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_setprio(0);
        }
    }
}

// Persistent batched sweep: many windows of many simulations in one launch.
// The work is the list of (step, packed item) pairs in step-major order; a
// wave takes `chunk` consecutive pairs from a 64-bit counter and runs them in
// order, with the per-job neighbour waits of the single-simulation persistent
// sweep (its epochs, coherent accesses and completion wait), plus a wait for
// the block's own previous window, which another wave may hold.  An item only
// waits for items earlier in the list, which were taken by running waves that
// run their own items in order, so the earliest unfinished item can always
// proceed: no co-residency of the grid is needed.
template <int P, int BX, int BY, int MODEL, int WPG>
__global__ __launch_bounds__(64 * WPG) void k_sweep_batched_persistent(BatchPersistArgs a)
{
    using C = Cfg<P, BX, BY, MODEL>;
    __shared__ __attribute__((aligned(16))) uint8_t lds[WPG * C::LDS];
    const int wid = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const uint64_t total = (uint64_t)(a.s1 - a.s0) * a.n_items;
    for (;;) {
        unsigned long long q0 = 0;
        if (lane == 0)
            q0 = atomicAdd(a.queue, (unsigned long long)a.chunk);
        q0 = __shfl(q0, 0, 64);
        if (q0 >= total)
            return;
        const uint64_t q1 = q0 + a.chunk < total ? q0 + a.chunk : total;
        for (uint64_t q = q0; q < q1; ++q) {
            const uint32_t s = a.s0 + (uint32_t)(q / a.n_items);
            const uint32_t it = (uint32_t)(q % a.n_items);
            const JobDesc& jd = a.jobs[a.item_job[it]];
            const uint64_t w = jd.base_window + s;
            if (w >= jd.n_windows)
                continue;
            const int c = jd.win_colour[w];
            const uint32_t k = it - jd.item_begin;
            const int beg = jd.colour_off[c], count = jd.colour_off[c + 1] - beg;
            if (k >= (uint32_t)count)
                continue;
            const int m = jd.blocks[beg + k];
            if (wait_neighbours(jd.nbr, jd.epoch, m, (int)w, lane, a.abort_flag, a.wait_ticks, true))
                return;
            __builtin_amdgcn_s_setprio(3); // as in the single-simulation persistent sweep
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            block_window<P, BX, BY, MODEL, true>(jd.lat, jd.table, jd.cnt, jd.Lx, jd.Ly, m, jd.NBX, jd.k0, jd.k1,
                                                 (uint32_t)w, jd.win_dur[w], lds + wid * C::LDS, false);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_s_waitcnt(0x0F70); // lattice stores performed before the epoch
            if (lane == 0) {
                const int nxt = jd.next_part[(size_t)c * (jd.n_windows + 1) + w + 1];
                __hip_atomic_store(&jd.epoch[m], nxt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __builtin_amdgcn_s_setprio(0);
        }
    }
}

// Epochs of every job of a batch at its current window: one workgroup per job.
__global__ void k_epoch_init_batched(const JobDesc* __restrict__ jobs)
{
    const JobDesc& jd = jobs[blockIdx.x];
    for (int m = threadIdx.x; m < jd.nb; m += blockDim.x)
        jd.epoch[m] = jd.next_part[(size_t)jd.bcol[m] * (jd.n_windows + 1) + jd.base_window];
}

// ---------------------------------------------------------------------------
// Resident persistent sweep (spin flip).  Wave g owns blocks g*bpw .. g*bpw +
// bpw-1 (bpw <= BPW; with bpw = 2 a horizontally adjacent pair, one block of
// each checkerboard colour, so the wave works in every window) for the whole
// launch and keeps their tiles in LDS; the lattice in HBM is read once at the
// start and written once at the end.  Between windows only the
// one-site boundary layers move (the local synchronisation of Sec. 2.2 stage
// 2): after each of its windows a block publishes its first/last row and
// first/last column as edge[4m + d] = tag | bits << 32 with one 64-bit
// agent-coherent store, tag = window + 1 (w0 for the state at the start of
// the launch).  Before block m runs window w it polls the four facing edges
// of its neighbours until each carries the tag of that neighbour's last
// window before w; data and tag travel in one single-copy-atomic word, so no
// fence or completion wait is needed.  A word is overwritten only after every
// reader of its previous value has published the edges its own window
// produced, which the writer's next window waits for.  Edges of blocks the
// same wave owns are read from the wave's LDS copy instead.  Waits are bounded
// (wait_ticks of the 100 MHz wall clock; then the abort flag is raised and
// every wave leaves without writing back).

// The P site states of a lane's segment as bits (site c0 + q in bit q), and back.
template <int P>
__device__ __forceinline__ uint32_t seg_bits(const Seg<P>& s)
{
    if constexpr (P == 1) {
        return s.w[0] & 1u;
    } else {
        // bit 0 of byte q moves to bit 24 + q: the product's terms below bit
        // 24 never share a position, so nothing carries into bits 24..27
        uint32_t b = 0;
#pragma unroll
        for (int k = 0; k < P / 4; ++k)
            b |= (((s.w[k] & 0x01010101u) * 0x01020408u) >> 24) << (4 * k);
        return b;
    }
}

template <int P>
__device__ __forceinline__ Seg<P> bits_seg(uint32_t b)
{
    Seg<P> s;
    if constexpr (P == 1) {
        s.w[0] = b & 1u;
    } else {
        // x * (1 + 2^7 + 2^14 + 2^21) holds copies of the 4-bit x at bit
        // offsets 0, 7, 14 and 21, which do not overlap; bit q of the copy at
        // 7q lands on bit 8q, the one bit of byte q the mask keeps
#pragma unroll
        for (int k = 0; k < P / 4; ++k)
            s.w[k] = (((b >> (4 * k)) & 0xFu) * 0x00204081u) & 0x01010101u;
    }
    return s;
}

// Publish the four boundary layers of the block in `tile` with tag `tag`.
// Rows: each lane puts its P bits at its column; an OR over the lanes of the
// row (quad DPP when a row is 2 or 4 lanes) leaves the row's bits in all of
// them.  Columns: lane i < BY fetches the masks of the first and last lane of
// row i (ds_bpermute), so one ballot per column gives its bits in order.
// mask: the lane's P site states as bits (site c0 + q in bit q).
template <int P, int BX, int BY>
__device__ __forceinline__ void publish_edges_bits(uint32_t mask, unsigned long long* edge, uint32_t* ledge,
                                                   uint32_t tag, int lane, int c0)
{
    using C = Cfg<P, BX, BY, MODEL_FLIP>;
    uint32_t e0 = 0, e1 = 0;
    if constexpr (C::DIM == 2) {
        if constexpr (C::LPR == 2 || C::LPR == 4) {
            uint32_t v = mask << c0;
            v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false); // quad_perm [1,0,3,2]
            if constexpr (C::LPR == 4)
                v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false); // quad_perm [2,3,0,1]
            e0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 0);
            e1 = (uint32_t)__builtin_amdgcn_readlane((int)v, (BY - 1) * C::LPR);
        } else {
#pragma unroll
            for (int j = 0; j < C::LPR; ++j) {
                e0 |= (uint32_t)__builtin_amdgcn_readlane((int)mask, j) << (j * P);
                e1 |= (uint32_t)__builtin_amdgcn_readlane((int)mask, (BY - 1) * C::LPR + j) << (j * P);
            }
        }
    }
    const int first = (lane % BY) * C::LPR;
    const uint32_t lm = (uint32_t)__builtin_amdgcn_ds_bpermute(4 * first, (int)mask);
    const uint32_t rm = (uint32_t)__builtin_amdgcn_ds_bpermute(4 * (first + C::LPR - 1), (int)mask);
    const uint32_t e2 = (uint32_t)__ballot(lane < BY && (lm & 1u));
    const uint32_t e3 = (uint32_t)__ballot(lane < BY && ((rm >> (P - 1)) & 1u));
    if (lane < 4) {
        const uint32_t bits = lane == 0 ? e0 : lane == 1 ? e1 : lane == 2 ? e2 : e3;
        coh_store(edge + lane, (unsigned long long)tag | ((unsigned long long)bits << 32));
        ledge[lane] = bits;
    }
}

template <int P, int BX, int BY>
__device__ __forceinline__ void publish_edges(const uint8_t* tile, int tb, unsigned long long* edge, uint32_t* ledge,
                                              uint32_t tag, int lane, int c0)
{
    publish_edges_bits<P, BX, BY>(seg_bits<P>(load_seg<P>(tile + tb)), edge, ledge, tag, lane, c0);
}

// Uniform reads of read-only per-window tables through the scalar cache
// (constant address space): a vector load in the resident window loop makes
// the next wait on a poll also wait for every earlier store, since loads and
// stores complete through one in-order counter.  The colour array is padded
// to whole dwords (scalar loads read dwords).
__device__ __forceinline__ int window_colour(const int8_t* wc, int w)
{
    const uint32_t d = *(const __attribute__((address_space(4))) uint32_t*)(uintptr_t)(wc + (w & ~3));
    return (int)(int8_t)(d >> (8 * (w & 3)));
}

__device__ __forceinline__ double window_length(const double* wd, int w)
{
    return *(const __attribute__((address_space(4))) double*)(uintptr_t)(wd + w);
}

template <int P, int BX, int BY, int WPG, int BPW>
__global__ __launch_bounds__(64 * WPG) void k_sweep_resident(ResidentArgs a)
{
    using C = Cfg<P, BX, BY, MODEL_FLIP>;
    constexpr int KMAX = 128; // colours tracked per wave (the library allows at most 127)
    constexpr int WAVE = (BPW * C::TILE + C::NTAB * 8 + C::XFER + 3 * BPW * 16 + KMAX * 4 + BPW * 16 + 15) / 16 * 16;
    __shared__ __attribute__((aligned(16))) uint8_t lds[WPG * WAVE];
    const int wid = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    uint8_t* wl = lds + wid * WAVE;
    double* tab = reinterpret_cast<double*>(wl + BPW * C::TILE);
    uint32_t* ledge = reinterpret_cast<uint32_t*>(wl + BPW * C::TILE + C::NTAB * 8 + C::XFER); // [BPW][4]
    // per owned block and poll lane d (0 above, 1 below, 2 left, 3 right):
    // the neighbour's block id, or -1 - i when this wave owns it as block i,
    // and the neighbour's colour; then per colour the last window of that
    // colour run so far in this launch (-1: none), so the tag a neighbour's
    // edge must carry is an LDS read instead of two dependent global loads
    int32_t* nbl = reinterpret_cast<int32_t*>(ledge + 4 * BPW); // [BPW][4]
    int32_t* ncl = nbl + 4 * BPW;                               // [BPW][4]
    int32_t* lastw = ncl + 4 * BPW;                             // [KMAX]
    // per owned block, the counter record's updates of this launch, written to
    // HBM once at its end: W of the block's last window (~0: not run), block-
    // windows with events, and events.  Written every window they would sit in
    // front of the next poll: loads and stores share one in-order counter, so
    // waiting for a poll's value also waits for every earlier store and atomic
    uint32_t* cwl = reinterpret_cast<uint32_t*>(lastw + KMAX); // [BPW][4]: W, writes, events lo, hi
    const int gw = __builtin_amdgcn_readfirstlane((int)xcd_order(blockIdx.x, gridDim.x) * WPG + wid);
    // the owner ranges through the scalar cache (uniform, read-only while the
    // kernel runs).  Read with a vector load, the value is pending on a path
    // the waitcnt pass cannot rule out, and every block-window then waits for
    // all outstanding vector memory operations (the previous window's edge
    // stores) before issuing its poll: 6.14 -> 6.04 ms on the headline run.
    int m0 = gw * a.bpw, want_own = a.bpw;
    if (a.owner) {
        const __attribute__((address_space(4))) int32_t* ow =
            (const __attribute__((address_space(4))) int32_t*)(uintptr_t)a.owner;
        m0 = ow[gw];
        want_own = ow[gw + 1] - m0;
    }
    const int r = lane / C::LPR, c0 = (lane % C::LPR) * P;
    const int tb = (r + 1) * C::S + P + c0;
    const size_t sLx = (size_t)a.Lx;

    for (int i = lane; i < C::NTAB; i += 64)
        tab[i] = a.table[i];
    int nown = 0;
    static_assert(BPW <= 8, "one colour byte per owned block");
    uint64_t cols = 0; // colour of owned block i in byte i
    for (int i = 0; i < want_own && i < BPW; ++i) {
        const int m = m0 + i;
        if (m >= a.nb)
            break;
        const int x0 = (m % a.NBX) * BX, y0 = (m / a.NBX) * BY;
        store_seg<P>(wl + i * C::TILE + tb, load_seg<P>(a.lat + (size_t)(y0 + r) * sLx + x0 + c0));
        cols |= (uint64_t)(uint8_t)a.bcol[m] << (8 * i);
        nown = i + 1;
    }
    // lanes 0..3 poll the facing edge (index dd) of the block above, below,
    // left, right
    const bool active = lane < 4 && (C::DIM == 2 || lane >= 2);
    const int dd = lane == 0 ? 1 : lane == 1 ? 0 : lane == 2 ? 3 : 2;
    for (int i = 0; i < nown; ++i) {
        if (active) {
            const int m = m0 + i;
            const int bi = m % a.NBX, bj = m / a.NBX;
            int nbm;
            if (lane == 0)
                nbm = (bj == 0 ? a.NBY - 1 : bj - 1) * a.NBX + bi;
            else if (lane == 1)
                nbm = (bj + 1 == a.NBY ? 0 : bj + 1) * a.NBX + bi;
            else if (lane == 2)
                nbm = bj * a.NBX + (bi == 0 ? a.NBX - 1 : bi - 1);
            else
                nbm = bj * a.NBX + (bi + 1 == a.NBX ? 0 : bi + 1);
            const bool local = nbm >= m0 && nbm < m0 + nown; // owned by this wave: LDS copy
            nbl[4 * i + lane] = local ? -1 - (nbm - m0) : nbm;
            ncl[4 * i + lane] = (uint8_t)a.bcol[nbm];
        }
    }
    for (int k = lane; k < KMAX; k += 64)
        lastw[k] = -1;
    if (lane < 4 * BPW)
        cwl[lane] = (lane & 3) == 0 ? ~0u : 0u;
    wave_sync();
#pragma unroll 1
    for (int i = 0; i < nown; ++i)
        publish_edges<P, BX, BY>(wl + i * C::TILE, tb, a.edge + 4 * (size_t)(m0 + i), ledge + 4 * i,
                                 (uint32_t)a.w0, lane, c0);

#pragma unroll 1
    for (int w = a.w0; w < a.w1; ++w) {
        const int c = window_colour(a.win_colour, w);
#pragma unroll 1
        for (int i = 0; i < nown; ++i) {
            if ((int)((cols >> (8 * i)) & 0xffu) != c)
                continue;
            const int m = m0 + i;
            uint8_t* tile = wl + i * C::TILE;
            // every lane issues the first poll (lanes that poll nothing read
            // their own block's edge word) and reads an LDS edge slot, so no
            // divergent branch surrounds the load; the values are joined
            // after the work below
            uint32_t want = 0;
            const int nb = active ? nbl[4 * i + lane] : -1;
            const bool remote = active && nb >= 0;
            const unsigned long long* src = a.edge + 4 * (size_t)(nb >= 0 ? nb : m) + (active ? dd : 0);
            const unsigned long long vg = coh_load(src);
            const unsigned long long vl = (unsigned long long)ledge[4 * (nb < 0 ? -1 - nb : 0) + (active ? dd : 0)] << 32;
            if (remote) {
                const int last = lastw[ncl[4 * i + lane]];
                want = last >= 0 ? (uint32_t)last + 1u : (uint32_t)a.w0;
            }
            // this lane's first draw of the window, the block's own rows and
            // the window's length, taken while the poll is in flight (the empty asm keeps the
            // compiler from sinking them below the wait); the halo cells read
            // here are replaced by the neighbours' edges after the wait
            const uint4 rr = philox10(make_uint4((uint32_t)lane, (uint32_t)m, (uint32_t)w, 0u), a.k0, a.k1);
            const double nl0 = -fs_log(unif_open0(rr));
            const double v0 = unif_open1(rr);
            FlipRows<P> g = flip_rows_from_tile<P, BY, C::S>(tile, tb);
            const double dur = window_length(a.win_dur, w);
            asm volatile("" ::"v"(nl0), "v"(v0), "v"(g.o.w[0]), "v"(g.lft), "v"(g.rgt), "v"(dur));
            unsigned long long v = remote ? vg : (active ? vl : 0ull);
            bool bad = false;
            if (active && nb >= 0 && (uint32_t)v != want) {
                const uint64_t t0 = wall_clock64();
                for (uint32_t n = 1;; ++n) {
                    __builtin_amdgcn_s_sleep(1);
                    v = coh_load(src);
                    if ((uint32_t)v == want)
                        break;
                    if ((n & 7u) == 0) { // the abort flag and the clock every eighth poll
                        if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            bad = true;
                            break;
                        }
                        if (wall_clock64() - t0 > a.wait_ticks) {
                            __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            bad = true;
                            break;
                        }
                    }
                }
            }
            if (__ballot(bad))
                return;
            // From here to the edge publication the wave is on its
            // neighbours' critical path; the other wave of the SIMD is then
            // usually drawing its next window's numbers or polling, work that
            // can wait: issue priority goes to this one (an A/B on the
            // headline: +6%, bits unchanged).
            __builtin_amdgcn_s_setprio(3);
            const uint32_t hv = (uint32_t)(v >> 32);
            const uint32_t top = (uint32_t)__builtin_amdgcn_readlane((int)hv, 0);
            const uint32_t bot = (uint32_t)__builtin_amdgcn_readlane((int)hv, 1);
            const uint32_t lft = (uint32_t)__builtin_amdgcn_readlane((int)hv, 2);
            const uint32_t rgt = (uint32_t)__builtin_amdgcn_readlane((int)hv, 3);
            if constexpr (C::DIM == 2) {
                if (r == 0)
                    g.dn = bits_seg<P>(top >> c0);
                if (r == BY - 1)
                    g.up = bits_seg<P>(bot >> c0);
            }
            if (c0 == 0)
                g.lft = (lft >> r) & 1u;
            if (c0 + P == BX)
                g.rgt = (rgt >> r) & 1u;
            FlipSites<P> F;
            flip_sites_from_rows<P, BY>(g, F);
            Seg<P> fo;

            const uint32_t e = ssa_window<P, BX, BY, MODEL_FLIP>(tile, tab, a.table, (uint32_t)m, (uint32_t)w, dur,
                                                                 a.k0, a.k1, true, nl0, v0, &F, true, &fo);
            // from the final sites in registers: the tile store completes at
            // the wave sync that ends the window
            // a window without events leaves the edges as they were: only the
            // tag moves, with the bits kept in LDS from the last publication
            if (e > 0) {
                publish_edges_bits<P, BX, BY>(seg_bits<P>(fo), a.edge + 4 * (size_t)m, ledge + 4 * i,
                                              (uint32_t)w + 1u, lane, c0);
            } else if (lane < 4) {
                coh_store(a.edge + 4 * (size_t)m + lane,
                          (unsigned long long)((uint32_t)w + 1u) | ((unsigned long long)ledge[4 * i + lane] << 32));
            }
            __builtin_amdgcn_s_setprio(0);
            if (lane == 0) {
                cwl[4 * i] = e;
                if (e > 0) {
                    cwl[4 * i + 1] += 1u;
                    unsigned long long* ev = reinterpret_cast<unsigned long long*>(cwl + 4 * i + 2);
                    *ev += e;
                }
            }
        }
        if (lane == 0)
            lastw[c] = w;
        wave_sync();
    }
    if (lane == 0) {
        for (int i = 0; i < nown; ++i) {
            const int m = m0 + i;
            if (cwl[4 * i] != ~0u)
                a.cnt[m].W = cwl[4 * i];
            if (cwl[4 * i + 1] != 0u) {
                atomicAdd(&a.cnt[m].writes, cwl[4 * i + 1]);
                atomicAdd(&a.cnt[m].events, *reinterpret_cast<const unsigned long long*>(cwl + 4 * i + 2));
            }
        }
    }
#pragma unroll 1
    for (int i = 0; i < nown; ++i) {
        const int m = m0 + i;
        const int x0 = (m % a.NBX) * BX, y0 = (m / a.NBX) * BY;
        store_seg<P>(a.lat + (size_t)(y0 + r) * sLx + x0 + c0, load_seg<P>(wl + i * C::TILE + tb));
    }
}

// ---------------------------------------------------------------------------
// Nested sweep (Sec. 5, eqs. sublatt2 and opdecomp2).  A coarse cell of C x C
// fine blocks is one workgroup; its tile (cell plus the one-site ring of the
// neighbouring cells, frozen for the outer window) is staged once into LDS.
// In every inner window the blocks of the active inner colour run their SSA
// windows concurrently, one wave each, on the shared tile: their neighbours in
// other fine blocks are plain LDS reads, and the workgroup barrier between
// inner windows is the only synchronisation.  At the end the cell (pair
// models: cell and ring) goes back to HBM.  Draws use the global block id and
// window index, so the result is the flat scheme's on the product colouring.
template <int P, int B, int MODEL, int CC, int KI>
struct NestCfg {
    using C = Cfg<P, B, B, MODEL>;
    static constexpr int WPG = CC * CC / KI;
    static constexpr int CS = CC * B;                            // cell side in sites
    static constexpr int TS = CS + 2 * P;                        // tile row stride
    static constexpr int TILE = ((CS + 2) * TS + 15) / 16 * 16;
    static constexpr int WAVE = (C::NTAB * 8 + C::XFER + 15) / 16 * 16; // per-wave table copy + exchange
    static constexpr int LDS = TILE + WPG * WAVE;
    static_assert(KI == 2 || KI == 4, "inner colourings: 2 (checkerboard) or 4");
    static_assert(CC % 2 == 0 && WPG <= 16, "cells of an even number of blocks, at most 16 waves");
};

// Position (lx, ly) in the cell of the j-th fine block of inner colour ci,
// for the inner colourings (lx+ly)%2 and (lx%2)+2(ly%2), row by row.
template <int CC, int KI>
__device__ __forceinline__ void nest_slot(int ci, int j, int& lx, int& ly)
{
    if constexpr (KI == 2) {
        ly = j / (CC / 2);
        lx = 2 * (j % (CC / 2)) + ((ly + ci) & 1);
    } else {
        ly = 2 * (j / (CC / 2)) + (ci >> 1);
        lx = 2 * (j % (CC / 2)) + (ci & 1);
    }
}

__device__ __forceinline__ int wrap(int v, int n)
{
    return v < 0 ? v + n : (v >= n ? v - n : v);
}

// Copy rows [r0, r1) (cell coordinates, -1 and CS are the ring) of the cell's
// interior columns between HBM and the tile, words where the layout allows.
template <int P, int TS, int CS, bool TO_LDS>
__device__ __forceinline__ void nest_rows(uint8_t* tile, uint8_t* lat, int Lx, int Ly, int x0, int y0, int r0, int r1,
                                          int tid, int nthr)
{
    if constexpr (P % 4 == 0) {
        constexpr int WR = CS / 4;
        for (int i = tid; i < (r1 - r0) * WR; i += nthr) {
            const int y = r0 + i / WR, x = 4 * (i % WR);
            uint32_t* g = reinterpret_cast<uint32_t*>(lat + (size_t)wrap(y0 + y, Ly) * Lx + x0 + x);
            uint32_t* t = reinterpret_cast<uint32_t*>(tile + (y + 1) * TS + P + x);
            if constexpr (TO_LDS)
                *t = *g;
            else
                *g = *t;
        }
    } else {
        for (int i = tid; i < (r1 - r0) * CS; i += nthr) {
            const int y = r0 + i / CS, x = i % CS;
            uint8_t* g = lat + (size_t)wrap(y0 + y, Ly) * Lx + x0 + x;
            uint8_t* t = tile + (y + 1) * TS + P + x;
            if constexpr (TO_LDS)
                *t = *g;
            else
                *g = *t;
        }
    }
}

// The ring columns -1 and CS of rows [0, CS).
template <int P, int TS, int CS, bool TO_LDS>
__device__ __forceinline__ void nest_cols(uint8_t* tile, uint8_t* lat, int Lx, int Ly, int x0, int y0, int tid,
                                          int nthr)
{
    for (int i = tid; i < 2 * CS; i += nthr) {
        const int y = i >> 1, x = (i & 1) ? CS : -1;
        uint8_t* g = lat + (size_t)wrap(y0 + y, Ly) * Lx + wrap(x0 + x, Lx);
        uint8_t* t = tile + (y + 1) * TS + P + x;
        if constexpr (TO_LDS)
            *t = *g;
        else
            *g = *t;
    }
}

template <int P, int B, int MODEL, int CC, int KI>
__global__ __launch_bounds__(64 * (CC * CC / KI)) void k_sweep_nested(NestedArgs a)
{
    using N = NestCfg<P, B, MODEL, CC, KI>;
    using C = Cfg<P, B, B, MODEL>;
    constexpr int NT = 64 * N::WPG;
    __shared__ __attribute__((aligned(16))) uint8_t lds[N::LDS];
    __shared__ int changed;
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    const int cell = a.cells[xcd_order(blockIdx.x, gridDim.x)];
    const int I = cell % a.NCX, J = cell / a.NCX;
    const int x0 = I * N::CS, y0 = J * N::CS;
    uint8_t* tile = lds;
    double* tab = reinterpret_cast<double*>(lds + N::TILE + wid * N::WAVE);
    for (int i = lane; i < C::NTAB; i += 64)
        tab[i] = (MODEL == MODEL_FLIP) ? a.table[i] : a.table[i * 14 + 13];
    if (tid == 0)
        changed = 0;
    nest_rows<P, N::TS, N::CS, true>(tile, a.lat, a.Lx, a.Ly, x0, y0, -1, N::CS + 1, tid, NT);
    nest_cols<P, N::TS, N::CS, true>(tile, a.lat, a.Lx, a.Ly, x0, y0, tid, NT);
    __syncthreads();

    uint32_t mine = 0;
    for (int w = a.w0; w < a.w1; ++w) {
        const int ci = (int)a.win_colour[w] % KI;
        int lx, ly;
        nest_slot<CC, KI>(ci, wid, lx, ly);
        const int m = (J * CC + ly) * a.NBX + I * CC + lx;
        uint8_t* sub = tile + ly * B * N::TS + lx * B;
        const uint32_t e =
            ssa_window<P, B, B, MODEL, N::TS>(sub, tab, a.table, (uint32_t)m, (uint32_t)w, a.win_dur[w], a.k0, a.k1);
        if (lane == 0) {
            a.cnt[m].W = e;
            if (e > 0) {
                atomicAdd(&a.cnt[m].writes, 1u);
                atomicAdd(&a.cnt[m].events, (unsigned long long)e);
            }
        }
        mine |= e;
        __syncthreads();
    }
    if (lane == 0 && mine)
        changed = 1;
    __syncthreads();
    if (!changed)
        return;
    if constexpr (MODEL == MODEL_FLIP) {
        nest_rows<P, N::TS, N::CS, false>(tile, a.lat, a.Lx, a.Ly, x0, y0, 0, N::CS, tid, NT);
    } else {
        nest_rows<P, N::TS, N::CS, false>(tile, a.lat, a.Lx, a.Ly, x0, y0, -1, N::CS + 1, tid, NT);
        nest_cols<P, N::TS, N::CS, false>(tile, a.lat, a.Lx, a.Ly, x0, y0, tid, NT);
    }
}

// Resident nested sweep (spin flip; Sec. 5 with the local synchronisation of
// Sec. 2.2 at the coarse level).  Every coarse cell is one workgroup for the
// whole launch and keeps its tile in LDS; the lattice is read once at the
// start and written once at the end.  The cell's four one-site boundary
// layers (4 x CS sites, listed top row, bottom row, left column, right
// column) are published as bits, 32 per 64-bit word tagged with the outer
// window just finished + 1 (ow0 at the start).  Before a cell runs its part
// of outer window k, wave 0 polls the words of its four neighbours that hold
// the layers facing it until each carries the tag of that neighbour's last
// outer window before k (same argument as the block-level resident sweep:
// tag and bits travel in one word, and a word is only overwritten after its
// readers have moved on), the ring is rebuilt from them, and the inner windows
// run as in the per-launch nested sweep.  Waits are bounded by wait_ticks.
template <int P, int B, int CC, int KI>
__global__ __launch_bounds__(64 * (CC * CC / KI)) void k_sweep_nested_resident(NestedResArgs a)
{
    using N = NestCfg<P, B, MODEL_FLIP, CC, KI>;
    using C = Cfg<P, B, B, MODEL_FLIP>;
    constexpr int NT = 64 * N::WPG;
    constexpr int CS = N::CS;
    constexpr int NE = 4 * CS;                 // boundary sites of a cell
    constexpr int NW = NE / 32;                // tagged words per cell
    constexpr int NWS = (CS + 31) / 32;        // words holding one side
    static_assert(NE % 64 == 0, "cells of at least 16 sites per side");
    __shared__ __attribute__((aligned(16))) uint8_t lds[N::LDS];
    __shared__ uint32_t ring[4 * NWS];         // polled words, per neighbour
    __shared__ int lastow[4];                  // last outer window of each outer colour, -1: none
    __shared__ int bad;
    // per block of the cell, the counter record's updates of this launch,
    // written to HBM once at its end (W of its last window, ~0: not run;
    // block-windows with events; events): written every inner window they
    // would sit in front of each barrier, which waits for every earlier store
    // and atomic
    __shared__ __attribute__((aligned(16))) uint32_t ncnt[CC * CC * 4];
    const int tid = threadIdx.x, wid = tid >> 6, lane = tid & 63;
    const int cell = (int)xcd_order(blockIdx.x, gridDim.x);
    const int I = cell % a.NCX, J = cell / a.NCX;
    const int x0 = I * CS, y0 = J * CS;
    auto outer_colour = [&](int i, int j) { return a.k_outer == 2 ? (i + j) % 2 : (i % 2) + 2 * (j % 2); };
    const int my = outer_colour(I, J);
    // neighbours above, below, left, right; the side of theirs that faces us
    const int nI[4] = {I, I, I == 0 ? a.NCX - 1 : I - 1, I + 1 == a.NCX ? 0 : I + 1};
    const int nJ[4] = {J == 0 ? a.NCY - 1 : J - 1, J + 1 == a.NCY ? 0 : J + 1, J, J};
    uint8_t* tile = lds;
    double* tab = reinterpret_cast<double*>(lds + N::TILE + wid * N::WAVE);
    for (int i = lane; i < C::NTAB; i += 64)
        tab[i] = a.table[i];
    if (tid < 4)
        lastow[tid] = -1;
    if (tid == 0)
        bad = 0;
    for (int t = tid; t < CC * CC * 4; t += NT)
        ncnt[t] = (t & 3) == 0 ? ~0u : 0u;
    nest_rows<P, N::TS, CS, true>(tile, a.lat, a.Lx, a.Ly, x0, y0, 0, CS, tid, NT);
    __syncthreads();

    // boundary site e (0 <= e < NE) of this cell in the tile
    auto edge_site = [&](int e) -> int {
        const int side = e / CS, pos = e % CS;
        const int y = side == 0 ? 0 : side == 1 ? CS - 1 : pos;
        const int x = side == 2 ? 0 : side == 3 ? CS - 1 : pos;
        return (y + 1) * N::TS + P + x;
    };
    auto publish = [&](uint32_t tag) {
        for (int k = wid; k < NE / 64; k += N::WPG) {
            const uint64_t bits = __ballot(tile[edge_site(64 * k + lane)] != 0);
            if (lane < 2)
                coh_store(a.edge + (size_t)cell * NW + 2 * k + lane,
                          (unsigned long long)tag | ((unsigned long long)(uint32_t)(bits >> (32 * lane)) << 32));
        }
    };
    publish((uint32_t)a.ow0);

    uint32_t mine = 0;
    // outer window bounds through the scalar cache: a vector load here would
    // wait for the previous outer window's edge stores
    const __attribute__((address_space(4))) int32_t* ofirst =
        (const __attribute__((address_space(4))) int32_t*)(uintptr_t)a.ofirst;
    for (int k = a.ow0; k < a.ow1; ++k) {
        const int wa = ofirst[k] > a.w0 ? ofirst[k] : a.w0;
        const int wb = ofirst[k + 1] < a.w1 ? ofirst[k + 1] : a.w1;
        const int co = window_colour(a.win_colour, wa) / KI;
        if (co == my) {
            // wave 0: lanes q*NWS + i poll word i of neighbour q's facing side
            if (wid == 0 && lane < 4 * NWS) {
                const int q = lane / NWS, i = lane % NWS;
                const int face = q == 0 ? 1 : q == 1 ? 0 : q == 2 ? 3 : 2;
                const int nc = nJ[q] * a.NCX + nI[q];
                const int last = lastow[outer_colour(nI[q], nJ[q])];
                const uint32_t want = last >= 0 ? (uint32_t)last + 1u : (uint32_t)a.ow0;
                const unsigned long long* src = a.edge + (size_t)nc * NW + (face * CS) / 32 + i;
                unsigned long long v = coh_load(src);
                if ((uint32_t)v != want) {
                    const uint64_t t0 = wall_clock64();
                    for (uint32_t n = 1;; ++n) {
                        __builtin_amdgcn_s_sleep(1);
                        v = coh_load(src);
                        if ((uint32_t)v == want)
                            break;
                        if ((n & 7u) == 0) {
                            if (__hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                                bad = 1;
                                break;
                            }
                            if (wall_clock64() - t0 > a.wait_ticks) {
                                __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                bad = 1;
                                break;
                            }
                        }
                    }
                }
                ring[lane] = (uint32_t)(v >> 32);
            }
            __syncthreads();
            if (bad)
                return; // uniform over the workgroup; nothing is written back
            // the ring from the polled words
            for (int r = tid; r < NE; r += NT) {
                const int q = r / CS, pos = r % CS;
                const int face = q == 0 ? 1 : q == 1 ? 0 : q == 2 ? 3 : 2;
                const int bit = face * CS + pos;
                const uint32_t v = (ring[q * NWS + (bit / 32 - (face * CS) / 32)] >> (bit % 32)) & 1u;
                const int y = q == 0 ? -1 : q == 1 ? CS : pos;
                const int x = q == 2 ? -1 : q == 3 ? CS : pos;
                tile[(y + 1) * N::TS + P + x] = (uint8_t)v;
            }
            __syncthreads();
            for (int w = wa; w < wb; ++w) {
                const int ci = window_colour(a.win_colour, w) % KI;
                int lx, ly;
                nest_slot<CC, KI>(ci, wid, lx, ly);
                const int m = (J * CC + ly) * a.NBX + I * CC + lx;
                uint8_t* sub = tile + ly * B * N::TS + lx * B;
                const uint32_t e = ssa_window<P, B, B, MODEL_FLIP, N::TS>(sub, tab, a.table, (uint32_t)m, (uint32_t)w,
                                                                          window_length(a.win_dur, w), a.k0, a.k1);
                if (lane == 0) {
                    uint32_t* r = ncnt + 4 * (ly * CC + lx);
                    r[0] = e;
                    if (e > 0) {
                        r[1] += 1u;
                        *reinterpret_cast<unsigned long long*>(r + 2) += e;
                    }
                }
                mine |= e;
                __syncthreads();
            }
            publish((uint32_t)k + 1u);
        }
        if (tid == 0)
            lastow[co] = k;
        __syncthreads();
    }
    (void)mine;
    __syncthreads();
    for (int bi = tid; bi < CC * CC; bi += NT) {
        const uint32_t* r = ncnt + 4 * bi;
        const int m = (J * CC + bi / CC) * a.NBX + I * CC + bi % CC;
        if (r[0] != ~0u)
            a.cnt[m].W = r[0];
        if (r[1] != 0u) {
            atomicAdd(&a.cnt[m].writes, r[1]);
            atomicAdd(&a.cnt[m].events, *reinterpret_cast<const unsigned long long*>(r + 2));
        }
    }
    nest_rows<P, N::TS, CS, false>(tile, a.lat, a.Lx, a.Ly, x0, y0, 0, CS, tid, NT);
}

// ---------------------------------------------------------------------------
// Block ranges of the next resident launch from the workload of the previous
// one (Sec. 6: the cumulative distribution of the workload histogram mapped
// onto equal masses over the processors), in one workgroup between launches.
// cost(m) = jumps of block m since the previous launch + base x (windows of
// its colour in that launch), or 1 for every block on the first launch; the
// costs' prefix sums C (C(0) = 0) give the quantile q_l = the first k with
// use * C(k) >= l * total (C(k) = k when the costs have no mass), clamped in
// order into [max(b_{l-1}, nb - (use-l) cap), min(b_{l-1} + cap, nb)].  With
// x_l = max(q_l, nb - (use-l) cap), which is non-decreasing and at most nb,
// that clamp is b_l = min(x_l, b_{l-1} + cap) = min over j <= l of
// x_j + (l-j) cap (x_0 = 0): a prefix minimum.  Waves use .. n_waves-1 get
// empty ranges.  ev_prev keeps the cumulative jump counts for the next call;
// scan holds nb prefix sums.
__global__ __launch_bounds__(1024) void k_rebalance(const BlockCount* cnt, unsigned long long* ev_prev,
                                                    const int8_t* bcol, const int8_t* win_colour, int pw0, int pw1,
                                                    int first, unsigned long long base, unsigned long long* scan,
                                                    int32_t* owner, int nb, int use, int n_waves, int cap)
{
    __shared__ unsigned long long part[1024];
    __shared__ long long pmin[1024];
    __shared__ unsigned int act[256];
    const int t = threadIdx.x;
    if (t < 256)
        act[t] = 0;
    __syncthreads();
    if (!first)
        for (int w = pw0 + t; w < pw1; w += 1024)
            atomicAdd(&act[(uint8_t)win_colour[w]], 1u);
    __syncthreads();
    const int chunk = (nb + 1023) / 1024;
    const int b0 = min(t * chunk, nb), b1 = min(b0 + chunk, nb);
    unsigned long long sum = 0;
    for (int m = b0; m < b1; ++m) {
        const unsigned long long ev = cnt[m].events;
        sum += first ? 1ull : ev - ev_prev[m] + base * act[(uint8_t)bcol[m]];
        ev_prev[m] = ev;
        scan[m] = sum; // prefix within the thread's run of blocks
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) { // inclusive scan of the run sums
        const unsigned long long v = t >= off ? part[t - off] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    const unsigned long long before = t > 0 ? part[t - 1] : 0ull, total = part[1023];
    for (int m = b0; m < b1; ++m)
        scan[m] += before; // C(m + 1)
    __syncthreads();
    for (int l = 1 + t; l < use; l += 1024) {
        int k;
        if (total == 0) {
            k = (int)(((long long)l * nb + use - 1) / use);
        } else {
            const unsigned __int128 target = (unsigned __int128)l * total;
            int lo = 0, hi = nb;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                const unsigned long long C = mid == 0 ? 0ull : scan[mid - 1];
                if ((unsigned __int128)C * (unsigned)use >= target)
                    hi = mid;
                else
                    lo = mid + 1;
            }
            k = lo;
        }
        owner[l] = k;
    }
    if (t == 0)
        owner[0] = 0;
    for (int l = use + t; l <= n_waves; l += 1024)
        owner[l] = nb;
    __syncthreads();
    // clamp: b_l = l cap + min over j <= l of (x_j - j cap), over runs of l
    const int lrun = (use + 1 + 1023) / 1024;
    const int l0 = min(t * lrun, use + 1), l1 = min(l0 + lrun, use + 1);
    constexpr long long kNone = 0x7fffffffffffffffll;
    long long run_min = kNone;
    for (int l = l0; l < l1; ++l) {
        const long long x = l == 0 ? 0ll : max((long long)owner[l], (long long)nb - (long long)(use - l) * cap);
        run_min = min(run_min, x - (long long)l * cap);
    }
    pmin[t] = run_min;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) { // inclusive prefix minimum of the run minima
        const long long v = t >= off ? pmin[t - off] : kNone;
        __syncthreads();
        pmin[t] = min(pmin[t], v);
        __syncthreads();
    }
    long long m = t > 0 ? pmin[t - 1] : kNone;
    for (int l = l0; l < l1; ++l) { // each thread reads and rewrites only its own run
        const long long x = l == 0 ? 0ll : max((long long)owner[l], (long long)nb - (long long)(use - l) * cap);
        m = min(m, x - (long long)l * cap);
        owner[l] = (int32_t)(m + (long long)l * cap);
    }
}

hipError_t launch_rebalance(const BlockCount* cnt, unsigned long long* ev_prev, const int8_t* bcol,
                            const int8_t* win_colour, int pw0, int pw1, int first, unsigned long long base,
                            unsigned long long* scan, int32_t* owner, int nb, int use, int n_waves, int cap,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_rebalance, dim3(1), dim3(1024), 0, s, cnt, ev_prev, bcol, win_colour, pw0, pw1, first, base,
                       scan, owner, nb, use, n_waves, cap);
    return hipGetLastError();
}

// epoch[m] = the first window >= w0 that block m takes part in.
__global__ void k_epoch_init(int32_t* epoch, const int8_t* bcol, const int32_t* next_part, int nb, int n_windows,
                             int w0)
{
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < nb; m += gridDim.x * blockDim.x)
        epoch[m] = next_part[bcol[m] * (n_windows + 1) + w0];
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
__global__ __launch_bounds__(256) void k_observe(const uint8_t* __restrict__ lat, int Lx, int Ly, int dim,
                                                 const BlockCount* __restrict__ cnt, int n_blocks,
                                                 unsigned long long* out)
{
    // per-thread counts fit 32 bits (at most 4 sites and 8 bonds per item,
    // at most 2^31 / 4 / (grid threads) items per thread); the wave and
    // workgroup sums are 64-bit, one global atomic per workgroup and counter
    __shared__ unsigned long long part[4][9];
    uint32_t acc[7] = {0, 0, 0, 0, 0, 0, 0};
    unsigned long long ev = 0, wr = 0;
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
            acc[0] += s == 0;
            acc[1] += s == 1;
            acc[2] += s == 2;
            acc[3] += s == 0 && rx == 0;
            acc[4] += s == 1 && rx == 1;
            acc[5] += s == 2 && rx == 2;
            acc[6] += (s == 1 && rx == 2) || (s == 2 && rx == 1);
            if (dim == 2) {
                const uint32_t ry = (up >> (8 * q)) & 0xffu;
                acc[3] += s == 0 && ry == 0;
                acc[4] += s == 1 && ry == 1;
                acc[5] += s == 2 && ry == 2;
                acc[6] += (s == 1 && ry == 2) || (s == 2 && ry == 1);
            }
        }
    }
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < n_blocks; b += stride) {
        ev += cnt[b].events;
        wr += cnt[b].writes;
    }
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        unsigned long long v = c < 7 ? (unsigned long long)acc[c] : (c == 7 ? ev : wr);
        for (int o = 32; o >= 1; o >>= 1)
            v += __shfl_xor(v, o, 64);
        if (lane == 0)
            part[wid][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        const unsigned long long v = part[0][threadIdx.x] + part[1][threadIdx.x] + part[2][threadIdx.x] +
                                     part[3][threadIdx.x];
        if (v)
            atomicAdd(out + threadIdx.x, v);
    }
}

// ---------------------------------------------------------------------------
// Dispatch.
template <typename K, typename... Args>
static hipError_t launch(K kernel, dim3 grid, dim3 block, hipStream_t s, LaunchTiming tm, Args... args)
{
    if (tm.start && tm.stop)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, tm.start, tm.stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    return hipGetLastError();
}

template <int MODEL, int WPG>
static hipError_t sweep_single_dispatch(int P, int shape, const SweepArgs& a, hipStream_t s, LaunchTiming tm)
{
    const dim3 grid((a.n_blocks + WPG - 1) / WPG), block(64 * WPG);
    if (shape == SHAPE_SQ) {
        if (P == 1)
            return launch(k_sweep_single<1, 8, 8, MODEL, WPG>, grid, block, s, tm, a);
        if (P == 4)
            return launch(k_sweep_single<4, 16, 16, MODEL, WPG>, grid, block, s, tm, a);
        if (P == 16)
            return a.n_blocks <= kLanePathBlocks
                       ? launch(k_sweep_single_lane<16, 32, 32, MODEL, WPG>, grid, block, s, tm, a)
                       : launch(k_sweep_single<16, 32, 32, MODEL, WPG>, grid, block, s, tm, a);
        return hipErrorInvalidValue;
    }
    if constexpr (MODEL != MODEL_FLIP) {
        return hipErrorInvalidValue;
    } else {
        if (P == 1)
            return launch(k_sweep_single<1, 64, 1, MODEL, WPG>, grid, block, s, tm, a);
        if (P == 4)
            return launch(k_sweep_single<4, 256, 1, MODEL, WPG>, grid, block, s, tm, a);
        if (P == 16)
            return a.n_blocks <= kLanePathBlocks
                       ? launch(k_sweep_single_lane<16, 1024, 1, MODEL, WPG>, grid, block, s, tm, a)
                       : launch(k_sweep_single<16, 1024, 1, MODEL, WPG>, grid, block, s, tm, a);
        return hipErrorInvalidValue;
    }
}

template <int MODEL, int WPG>
static hipError_t sweep_batched_dispatch(int P, int shape, const JobDesc* jobs, const uint32_t* item_job,
                                         uint32_t n_items, uint64_t step, hipStream_t s, LaunchTiming tm)
{
    const dim3 grid((n_items + WPG - 1) / WPG), block(64 * WPG);
    if (shape == SHAPE_SQ) {
        if (P == 1)
            return launch(k_sweep_batched<1, 8, 8, MODEL, WPG>, grid, block, s, tm, jobs, item_job, n_items, step);
        if (P == 4)
            return launch(k_sweep_batched<4, 16, 16, MODEL, WPG>, grid, block, s, tm, jobs, item_job, n_items, step);
        if (P == 16)
            return n_items <= (uint32_t)kLanePathBlocks
                       ? launch(k_sweep_batched_lane<16, 32, 32, MODEL, WPG>, grid, block, s, tm, jobs, item_job,
                                n_items, step)
                       : launch(k_sweep_batched<16, 32, 32, MODEL, WPG>, grid, block, s, tm, jobs, item_job, n_items,
                                step);
        return hipErrorInvalidValue;
    }
    if constexpr (MODEL != MODEL_FLIP) {
        return hipErrorInvalidValue;
    } else {
        if (P == 1)
            return launch(k_sweep_batched<1, 64, 1, MODEL, WPG>, grid, block, s, tm, jobs, item_job, n_items, step);
        if (P == 4)
            return launch(k_sweep_batched<4, 256, 1, MODEL, WPG>, grid, block, s, tm, jobs, item_job, n_items, step);
        if (P == 16)
            return n_items <= (uint32_t)kLanePathBlocks
                       ? launch(k_sweep_batched_lane<16, 1024, 1, MODEL, WPG>, grid, block, s, tm, jobs, item_job,
                                n_items, step)
                       : launch(k_sweep_batched<16, 1024, 1, MODEL, WPG>, grid, block, s, tm, jobs, item_job,
                                n_items, step);
        return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_single(int model, int P, int shape, int wpg, const SweepArgs& a, hipStream_t s,
                               LaunchTiming tm)
{
    if (a.n_blocks <= 0)
        return hipSuccess;
#define FSKMC_SW(MOD)                                                          \
    switch (wpg) {                                                             \
    case 1: return sweep_single_dispatch<MOD, 1>(P, shape, a, s, tm);          \
    case 2: return sweep_single_dispatch<MOD, 2>(P, shape, a, s, tm);          \
    case 4: return sweep_single_dispatch<MOD, 4>(P, shape, a, s, tm);          \
    case 8: return sweep_single_dispatch<MOD, 8>(P, shape, a, s, tm);          \
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
                                uint32_t n_items, uint64_t step, hipStream_t s, LaunchTiming tm)
{
    if (n_items == 0)
        return hipSuccess;
#define FSKMC_SW(MOD)                                                                            \
    switch (wpg) {                                                                               \
    case 1: return sweep_batched_dispatch<MOD, 1>(P, shape, jobs, item_job, n_items, step, s, tm); \
    case 2: return sweep_batched_dispatch<MOD, 2>(P, shape, jobs, item_job, n_items, step, s, tm); \
    case 4: return sweep_batched_dispatch<MOD, 4>(P, shape, jobs, item_job, n_items, step, s, tm); \
    case 8: return sweep_batched_dispatch<MOD, 8>(P, shape, jobs, item_job, n_items, step, s, tm); \
    default: return hipErrorInvalidValue;                                                        \
    }
    if (model == MODEL_FLIP) {
        FSKMC_SW(MODEL_FLIP)
    } else {
        FSKMC_SW(MODEL_ZGB)
    }
#undef FSKMC_SW
}

// Workgroups of a kernel that can be resident at once on the device
// (occupancy x CUs), cached per kernel; 0 when the runtime cannot say.
template <typename K>
static unsigned resident_grid(K kern, int threads)
{
    static std::vector<std::pair<const void*, unsigned>> cache;
    for (auto& e : cache)
        if (e.first == reinterpret_cast<const void*>(kern))
            return e.second;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    cache.emplace_back(reinterpret_cast<const void*>(kern), (unsigned)(per_cu * cus));
    return (unsigned)(per_cu * cus);
}

// grid == 0: as many workgroups as can be resident (the work counter spreads
// the items; more workgroups would only queue in the dispatcher)
template <typename K>
static hipError_t batched_persistent_launch(K kern, unsigned grid, int wpg, hipStream_t s, LaunchTiming tm,
                                            const BatchPersistArgs& a)
{
    if (grid == 0)
        grid = resident_grid(kern, 64 * wpg);
    if (grid == 0)
        grid = (unsigned)std::max(1, 2048 / wpg);
    return launch(kern, dim3(grid), dim3(64 * wpg), s, tm, a);
}

template <int MODEL, int WPG>
static hipError_t batched_persistent_dispatch(int P, int shape, const BatchPersistArgs& a, unsigned grid,
                                              hipStream_t s, LaunchTiming tm)
{
    if (shape == SHAPE_SQ) {
        switch (P) {
        case 1: return batched_persistent_launch(k_sweep_batched_persistent<1, 8, 8, MODEL, WPG>, grid, WPG, s, tm, a);
        case 4:
            return batched_persistent_launch(k_sweep_batched_persistent<4, 16, 16, MODEL, WPG>, grid, WPG, s, tm, a);
        case 16:
            return batched_persistent_launch(k_sweep_batched_persistent<16, 32, 32, MODEL, WPG>, grid, WPG, s, tm, a);
        }
    } else if constexpr (MODEL == MODEL_FLIP) {
        switch (P) {
        case 1: return batched_persistent_launch(k_sweep_batched_persistent<1, 64, 1, MODEL, WPG>, grid, WPG, s, tm, a);
        case 4:
            return batched_persistent_launch(k_sweep_batched_persistent<4, 256, 1, MODEL, WPG>, grid, WPG, s, tm, a);
        case 16:
            return batched_persistent_launch(k_sweep_batched_persistent<16, 1024, 1, MODEL, WPG>, grid, WPG, s, tm,
                                             a);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_sweep_batched_persistent(int model, int P, int shape, int wpg, const BatchPersistArgs& a,
                                           unsigned grid, hipStream_t s, LaunchTiming tm)
{
    if (a.chunk == 0 || a.s1 <= a.s0)
        return hipErrorInvalidValue;
    if (model == MODEL_FLIP) {
        switch (wpg) {
        case 1: return batched_persistent_dispatch<MODEL_FLIP, 1>(P, shape, a, grid, s, tm);
        case 2: return batched_persistent_dispatch<MODEL_FLIP, 2>(P, shape, a, grid, s, tm);
        case 4: return batched_persistent_dispatch<MODEL_FLIP, 4>(P, shape, a, grid, s, tm);
        case 8: return batched_persistent_dispatch<MODEL_FLIP, 8>(P, shape, a, grid, s, tm);
        }
    } else {
        switch (wpg) {
        case 1: return batched_persistent_dispatch<MODEL_ZGB, 1>(P, shape, a, grid, s, tm);
        case 2: return batched_persistent_dispatch<MODEL_ZGB, 2>(P, shape, a, grid, s, tm);
        case 4: return batched_persistent_dispatch<MODEL_ZGB, 4>(P, shape, a, grid, s, tm);
        case 8: return batched_persistent_dispatch<MODEL_ZGB, 8>(P, shape, a, grid, s, tm);
        }
    }
    return hipErrorInvalidValue;
}

unsigned batched_persistent_grid(int P, int shape, int wpg)
{
    (void)P;
    (void)shape;
    // a lower bound of the resident workgroups (256 CUs x 8 waves) for the
    // work-chunk size; the launch itself fills the device
    return (unsigned)std::max(1, 2048 / std::max(wpg, 1));
}

hipError_t launch_epoch_init_batched(const JobDesc* jobs, int n_jobs, hipStream_t s)
{
    if (n_jobs <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_epoch_init_batched, dim3(n_jobs), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

// Cooperative launch of the persistent sweep: as many workgroups as can be
// resident at once (occupancy x CUs), but no more than the largest colour
// class needs.
template <int P, int BX, int BY, int MODEL, int WPG>
static hipError_t persist_launch(PersistArgs a, int max_blocks_per_colour, hipStream_t s, LaunchTiming tm)
{
    auto kern = k_sweep_persistent<P, BX, BY, MODEL, WPG>;
    static int resident_groups = 0;
    if (resident_groups == 0) {
        int per_cu = 0, dev = 0, cus = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * WPG, 0);
        if (e != hipSuccess)
            return e;
        if ((e = hipGetDevice(&dev)) != hipSuccess ||
            (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
            return e;
        resident_groups = per_cu * cus;
        if (resident_groups <= 0)
            return hipErrorInvalidConfiguration;
    }
    const int want = (max_blocks_per_colour + WPG - 1) / WPG;
    const int groups = want < resident_groups ? want : resident_groups;
    a.n_waves = groups * WPG;
    void* args[] = {&a};
    if (tm.start)
        (void)hipEventRecord(tm.start, s);
    hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(groups), dim3(64 * WPG),
                                              args, 0, s);
    if (tm.stop)
        (void)hipEventRecord(tm.stop, s);
    return e;
}

// Cooperative launch of the resident sweep: an adjacent block pair per wave,
// more blocks per wave (up to res_bpw) when the lattice has more blocks than
// twice the resident waves, or the caller's ranges (owner array, one range
// per resident wave).
constexpr int res_bpw(int P) { return P == 16 ? 4 : 8; }

template <int P, int BX, int BY, int WPG>
static int resident_groups_of()
{
    auto kern = k_sweep_resident<P, BX, BY, WPG, res_bpw(P)>;
    static int resident_groups = 0;
    if (resident_groups == 0) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * WPG, 0) != hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0; // no resident launch possible: the caller streams
        resident_groups = per_cu * cus;
    }
    return resident_groups;
}

template <int P, int BX, int BY, int WPG>
static hipError_t resident_launch(ResidentArgs a, hipStream_t s, LaunchTiming tm)
{
    auto kern = k_sweep_resident<P, BX, BY, WPG, res_bpw(P)>;
    const int resident_groups = resident_groups_of<P, BX, BY, WPG>();
    if (resident_groups <= 0)
        return hipErrorInvalidConfiguration;
    if (a.nb <= 0)
        return hipErrorInvalidValue;
    int groups = 0;
    if (a.owner) {
        if (a.n_waves != resident_groups * WPG)
            return hipErrorInvalidValue;
        groups = resident_groups;
        a.bpw = 0;
    } else {
        // two blocks per wave (an adjacent pair of the two colours), more when
        // the lattice has more blocks than twice the resident waves
        const int cap = resident_groups * WPG;
        int bpw = a.nb >= 2 ? 2 : 1;
        if (bpw * cap < a.nb)
            bpw = (a.nb + cap - 1) / cap;
        if (bpw > res_bpw(P))
            return hipErrorInvalidConfiguration;
        a.bpw = bpw;
        const int waves = (a.nb + bpw - 1) / bpw;
        groups = (waves + WPG - 1) / WPG;
        a.n_waves = groups * WPG;
    }
    void* args[] = {&a};
    if (tm.start)
        (void)hipEventRecord(tm.start, s);
    hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(groups), dim3(64 * WPG),
                                              args, 0, s);
    if (tm.stop)
        (void)hipEventRecord(tm.stop, s);
    return e;
}

template <int WPG>
static hipError_t resident_dispatch(int P, int shape, const ResidentArgs& a, hipStream_t s, LaunchTiming tm)
{
    if (shape == SHAPE_SQ) {
        if (P == 1)
            return resident_launch<1, 8, 8, WPG>(a, s, tm);
        if (P == 4)
            return resident_launch<4, 16, 16, WPG>(a, s, tm);
        if (P == 16)
            return resident_launch<16, 32, 32, WPG>(a, s, tm);
        return hipErrorInvalidValue;
    }
    if (P == 1)
        return resident_launch<1, 64, 1, WPG>(a, s, tm);
    if (P == 4)
        return resident_launch<4, 256, 1, WPG>(a, s, tm);
    if (P == 16)
        return resident_launch<16, 1024, 1, WPG>(a, s, tm);
    return hipErrorInvalidValue;
}

hipError_t launch_sweep_resident(int P, int shape, int wpg, const ResidentArgs& a, hipStream_t s, LaunchTiming tm)
{
    return wpg == 1 ? resident_dispatch<1>(P, shape, a, s, tm) : resident_dispatch<2>(P, shape, a, s, tm);
}

template <int WPG>
static int resident_waves_of(int P, int shape)
{
    int g = 0;
    if (shape == SHAPE_SQ)
        g = P == 1 ? resident_groups_of<1, 8, 8, WPG>() : P == 4 ? resident_groups_of<4, 16, 16, WPG>()
                                                                 : resident_groups_of<16, 32, 32, WPG>();
    else
        g = P == 1 ? resident_groups_of<1, 64, 1, WPG>() : P == 4 ? resident_groups_of<4, 256, 1, WPG>()
                                                                  : resident_groups_of<16, 1024, 1, WPG>();
    return g * WPG;
}

int resident_waves(int P, int shape, int wpg)
{
    return wpg == 1 ? resident_waves_of<1>(P, shape) : resident_waves_of<2>(P, shape);
}

int resident_capacity(int P) { return res_bpw(P); }

template <int MODEL, int WPG>
static hipError_t persist_dispatch(int P, int shape, const PersistArgs& a, int maxpc, hipStream_t s, LaunchTiming tm)
{
    if (shape == SHAPE_SQ) {
        if (P == 1)
            return persist_launch<1, 8, 8, MODEL, WPG>(a, maxpc, s, tm);
        if (P == 4)
            return persist_launch<4, 16, 16, MODEL, WPG>(a, maxpc, s, tm);
        if (P == 16)
            return persist_launch<16, 32, 32, MODEL, WPG>(a, maxpc, s, tm);
        return hipErrorInvalidValue;
    }
    if constexpr (MODEL != MODEL_FLIP) {
        return hipErrorInvalidValue;
    } else {
        if (P == 1)
            return persist_launch<1, 64, 1, MODEL, WPG>(a, maxpc, s, tm);
        if (P == 4)
            return persist_launch<4, 256, 1, MODEL, WPG>(a, maxpc, s, tm);
        if (P == 16)
            return persist_launch<16, 1024, 1, MODEL, WPG>(a, maxpc, s, tm);
        return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_persistent(int model, int P, int shape, int wpg, const PersistArgs& a,
                                   int max_blocks_per_colour, hipStream_t s, LaunchTiming tm)
{
#define FSKMC_SW(MOD)                                                                    \
    switch (wpg) {                                                                       \
    case 1: return persist_dispatch<MOD, 1>(P, shape, a, max_blocks_per_colour, s, tm); \
    case 2: return persist_dispatch<MOD, 2>(P, shape, a, max_blocks_per_colour, s, tm); \
    case 4: return persist_dispatch<MOD, 4>(P, shape, a, max_blocks_per_colour, s, tm); \
    case 8: return persist_dispatch<MOD, 8>(P, shape, a, max_blocks_per_colour, s, tm); \
    default: return hipErrorInvalidValue;                                                \
    }
    if (model == MODEL_FLIP) {
        FSKMC_SW(MODEL_FLIP)
    } else {
        FSKMC_SW(MODEL_ZGB)
    }
#undef FSKMC_SW
}

template <int MODEL, int CC, int KI>
static hipError_t nested_p(int P, const NestedArgs& a, hipStream_t s, LaunchTiming tm)
{
    constexpr int T = 64 * (CC * CC / KI);
    switch (P) {
    case 1: return launch(k_sweep_nested<1, 8, MODEL, CC, KI>, dim3(a.n_cells), dim3(T), s, tm, a);
    case 4: return launch(k_sweep_nested<4, 16, MODEL, CC, KI>, dim3(a.n_cells), dim3(T), s, tm, a);
    case 16: return launch(k_sweep_nested<16, 32, MODEL, CC, KI>, dim3(a.n_cells), dim3(T), s, tm, a);
    default: return hipErrorInvalidValue;
    }
}

template <int CC, int KI>
static hipError_t nested_resident_p(int P, const NestedResArgs& a, hipStream_t s, LaunchTiming tm)
{
    constexpr int T = 64 * (CC * CC / KI);
    const void* kern = nullptr;
    switch (P) {
    case 1: kern = reinterpret_cast<const void*>(k_sweep_nested_resident<1, 8, CC, KI>); break;
    case 4: kern = reinterpret_cast<const void*>(k_sweep_nested_resident<4, 16, CC, KI>); break;
    case 16: kern = reinterpret_cast<const void*>(k_sweep_nested_resident<16, 32, CC, KI>); break;
    default: return hipErrorInvalidValue;
    }
    const unsigned cells = (unsigned)(a.NCX * a.NCY);
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, T, 0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        (unsigned)(per_cu * cus) < cells)
        return hipErrorInvalidConfiguration;
    NestedResArgs args = a;
    void* pa[] = {&args};
    if (tm.start)
        (void)hipEventRecord(tm.start, s);
    const hipError_t e = hipLaunchCooperativeKernel(kern, dim3(cells), dim3(T), pa, 0, s);
    if (tm.stop)
        (void)hipEventRecord(tm.stop, s);
    return e;
}

hipError_t launch_sweep_nested_resident(int P, int c, int k_inner, const NestedResArgs& a, hipStream_t s,
                                        LaunchTiming tm)
{
    if (!nested_supported(MODEL_FLIP, P, c, k_inner) || a.w1 <= a.w0 || a.ow1 <= a.ow0)
        return hipErrorInvalidValue;
    if (c == 2)
        return nested_resident_p<2, 2>(P, a, s, tm);
    return k_inner == 2 ? nested_resident_p<4, 2>(P, a, s, tm) : nested_resident_p<4, 4>(P, a, s, tm);
}

bool nested_supported(int model, int P, int c, int k_inner)
{
    if (P != 1 && P != 4 && P != 16)
        return false;
    if (model == MODEL_FLIP)
        return (c == 2 && k_inner == 2) || (c == 4 && (k_inner == 2 || k_inner == 4));
    return k_inner == 4 && (c == 2 || c == 4);
}

hipError_t launch_sweep_nested(int model, int P, int c, int k_inner, const NestedArgs& a, hipStream_t s,
                               LaunchTiming tm)
{
    if (!nested_supported(model, P, c, k_inner) || a.n_cells <= 0 || a.w1 <= a.w0)
        return hipErrorInvalidValue;
    if (model == MODEL_FLIP) {
        if (c == 2)
            return nested_p<MODEL_FLIP, 2, 2>(P, a, s, tm);
        return k_inner == 2 ? nested_p<MODEL_FLIP, 4, 2>(P, a, s, tm) : nested_p<MODEL_FLIP, 4, 4>(P, a, s, tm);
    }
    return c == 2 ? nested_p<MODEL_ZGB, 2, 4>(P, a, s, tm) : nested_p<MODEL_ZGB, 4, 4>(P, a, s, tm);
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

hipError_t launch_epoch_init(int32_t* epoch, const int8_t* bcol, const int32_t* next_part, int nb, int n_windows,
                             int w0, hipStream_t s)
{
    hipLaunchKernelGGL(k_epoch_init, dim3(grid_for(nb, 256)), dim3(256), 0, s, epoch, bcol, next_part, nb, n_windows,
                       w0);
    return hipGetLastError();
}

hipError_t launch_observe(const uint8_t* lat, int Lx, int Ly, int dim, const BlockCount* cnt, int n_blocks,
                          unsigned long long* out9, hipStream_t s)
{
    const int64_t work = std::max<int64_t>((int64_t)Lx * Ly / 4, n_blocks);
    unsigned g = grid_for(work, 256);
    if (g > 256)
        g = 256; // one workgroup per CU: 256 x 9 atomics per call
    hipLaunchKernelGGL(k_observe, dim3(g), dim3(256), 0, s, lat, Lx, Ly, dim, cnt, n_blocks, out9);
    return hipGetLastError();
}

}  // namespace fskmc
