/*
 * fskmc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU reference ("the oracle") for the
 * fractional-step lattice kinetic Monte Carlo method of Arampatzis,
 * Katsoulakis, Plechac, Taufer and Xu, "Hierarchical fractional-step
 * approximations and parallel kinetic Monte Carlo algorithms".
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this code.  It shares no source with the HIP library:
 * the Philox generator, the logarithm, the rates, the sum tree, the block
 * decomposition and the schedule are all written out again here.
 *
 * Two parts:
 *   (a) or_ssa_serial: the exact serial stochastic simulation algorithm of the
 *       whole-lattice continuous-time Markov chain, built from the total rate
 *       (Sec. 1, eq. totalrate) and the jump probabilities (eq. skeleton) of
 *       the generator (Sec. 2, eq. generator).
 *   (b) or_fs_run: the fractional-step scheme (Sec. 2.2, eqs. lie / exact and
 *       the three-stage step; Sec. 3, eqs. strang / PCSl / PCSs), run block by
 *       block: in each window every block of the active colour runs its own
 *       serial SSA kernel for the window's duration while everything else is
 *       frozen.  Its arithmetic follows the fixed contract that the GPU path
 *       reproduces bit for bit (FP64 pairwise sum tree in heap order, Philox
 *       counter layout, own logarithm, strict window boundary).
 *
 * Compile with -ffp-contract=off and without fast-math: the results depend on
 * IEEE round-to-nearest for +, -, *, / and on no fused multiply-add.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* Test hook: OR_PLANT selects one deliberate mistake; tests/test_oracle_plants.py
 * builds such variants to show that the pins catch each of them.  It is 0 in
 * every real build. */
#ifndef OR_PLANT
#define OR_PLANT 0
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_EDECOMP (-4)

#define OR_MODEL_FLIP 1
#define OR_MODEL_ZGB 2
#define OR_MODEL_KAW 3

#define OR_LIE 0
#define OR_STRANG 1
#define OR_RANDOM 2

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator, from its published definition
 * (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11): ten rounds of two 32x32->64 multiplications with the constants
 * 0xD2511F53 / 0xCD9E8D57 and a Weyl key schedule 0x9E3779B9 / 0xBB67AE85.    */
static void or_mulhilo(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < 10; round++) {
        uint32_t hi0, lo0, hi1, lo1;
        if (round > 0 || OR_PLANT == 2) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        or_mulhilo(0xD2511F53u, x0, &hi0, &lo0);
        or_mulhilo(0xCD9E8D57u, x2, &hi1, &lo1);
        {
            uint32_t y0 = hi1 ^ x1 ^ k0;
            uint32_t y1 = lo1;
            uint32_t y2 = hi0 ^ x3 ^ k1;
            uint32_t y3 = lo0;
            x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        }
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Two doubles from one Philox block: U in (0,1] from words 0,1 and V in [0,1)
 * from words 2,3, each the top 53 bits of a 64-bit word times 2^-53.         */
void or_uniforms(const uint32_t r[4], double* U, double* V)
{
    uint64_t a = ((uint64_t)r[0] << 32) | (uint64_t)r[1];
    uint64_t b = ((uint64_t)r[2] << 32) | (uint64_t)r[3];
    *U = (double)((a >> 11) + 1u) * 0x1p-53;
    *V = (double)(b >> 11) * 0x1p-53;
}

static void or_draw(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                    uint32_t seed, uint32_t replica, double* U, double* V)
{
    uint32_t ctr[4], key[2], r[4];
    ctr[0] = c0; ctr[1] = c1; ctr[2] = c2; ctr[3] = c3;
    key[0] = seed; key[1] = replica;
    or_philox(ctr, key, r);
    or_uniforms(r, U, V);
}

/* ------------------------------------------------------------------------ */
/* Natural logarithm from IEEE +,-,*,/ only, for u > 0 (here u in (0,1]).
 * u = m * 2^e with m in [sqrt(1/2), sqrt(2)); with s = (m-1)/(m+1),
 * log m = 2s (1 + z/3 + z^2/5 + ... ), z = s^2 (the atanh series), truncated
 * after the z^10/21 term, then log u = e*ln2_hi + (e*ln2_lo + log m) with
 * ln 2 split so that e*ln2_hi is exact.                                      */
static const double OR_LN2_HI = 0x1.62e42ff000000p-1;
static const double OR_LN2_LO = (OR_PLANT == 8 ? 1.0 : -1.0) * 0x1.718432a1b0e26p-35;
static const double OR_SQRT2 = 0x1.6a09e667f3bcdp+0;

double or_log(double u)
{
    uint64_t bits, mbits;
    int e;
    double m, f, s, z, P, two_s, logm;
    int k;
    memcpy(&bits, &u, 8);
    e = (int)((bits >> 52) & 0x7ffu);
    if (e == 0) { /* subnormal input: scale into the normal range first */
        u = u * 0x1p54;
        memcpy(&bits, &u, 8);
        e = (int)((bits >> 52) & 0x7ffu) - 54;
    }
    e -= 1023;
    mbits = (bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
    memcpy(&m, &mbits, 8); /* m in [1,2) */
    if (m >= OR_SQRT2) {
        m = m * 0.5;
        e = e + 1;
    }
    f = m - 1.0;
    s = f / (2.0 + f);
    z = s * s;
    P = 1.0 / 21.0; /* coefficient of z^9: 1/(2*10+1) */
    for (k = 9; k >= 1; k--)
        P = P * z + 1.0 / (double)(2 * k + 1);
    two_s = s + s;
    logm = two_s + two_s * (z * P);
    return (double)e * OR_LN2_HI + ((double)e * OR_LN2_LO + logm);
}

/* ------------------------------------------------------------------------ */
/* Models: lattice, spin space and the rates c(x, omega; sigma).
 * Sites are indexed y*Lx + x on a periodic Lx x Ly lattice (Ly = 1 in 1D).
 * Directions: d=0 (+x), d=1 (-x), d=2 (+y), d=3 (-y); 1D uses d=0,1.        */
typedef struct {
    int model;   /* OR_MODEL_FLIP, OR_MODEL_ZGB or OR_MODEL_KAW */
    int dim;     /* 1 or 2 */
    int Lx, Ly;
    double p[5]; /* flip: k_a, k_d, J, h, beta.  zgb: y, k_r, D.  kaw: D, J, beta */
} or_model;

static int or_ndir(const or_model* M) { return M->dim == 1 ? 2 : 4; }

static int or_neighbour(const or_model* M, int site, int d)
{
    int x = site % M->Lx, y = site / M->Lx;
    switch (d) {
    case 0: x = (x + 1) % M->Lx; break;
    case 1: x = (x - 1 + M->Lx) % M->Lx; break;
    case 2: y = (y + 1) % M->Ly; break;
    default: y = OR_PLANT == 5 ? (y + 1) % M->Ly : (y - 1 + M->Ly) % M->Ly; break;
    }
    return y * M->Lx + x;
}

/* Spin-flip Arrhenius adsorption/desorption (Sec. 4.1 eqs. adsdesrate and
 * potential; Sec. 7 eq. Arrhenius): c = k_a if sigma(x)=0 and
 * k_d exp(-beta (J * #occupied neighbours + h)) if sigma(x)=1.              */
static double or_flip_rate(const or_model* M, const uint8_t* lat, int site)
{
    int n = 0, d;
    for (d = 0; d < or_ndir(M); d++)
        n += lat[or_neighbour(M, site, d)];
    if (lat[site] == 0)
        return M->p[0];
    if (OR_PLANT == 1)
        return M->p[1] * exp(M->p[4] * (M->p[2] * (double)n + M->p[3]));
    return M->p[1] * exp(-(M->p[4] * (M->p[2] * (double)n + M->p[3])));
}

/* ZGB-type reaction model (Sec. 7.1, Table COrates) with states 0 empty,
 * 1 = A (monomer), 2 = B (fragment of the dimer).  Channels per site x, in
 * this order, one per neighbour direction d where a partner is involved:
 *   ch0      A adsorption            sigma(x)=0                     rate y
 *   ch1+d    B2 dissociative ads.    sigma(x)=sigma(x+e_d)=0        (1-y)/4
 *   ch5+d    A+B reaction -> 0,0     {sigma(x),sigma(x+e_d)}={A,B}  k_r/4
 *   ch9+d    A hop x -> x+e_d        sigma(x)=A, sigma(x+e_d)=0     D/4      */
#define OR_ZGB_NCH 13
static void or_zgb_channels(const or_model* M, const uint8_t* lat, int site, double ch[OR_ZGB_NCH])
{
    double y = M->p[0], kr = M->p[1], D = M->p[2];
    int s = lat[site], d;
    for (d = 0; d < OR_ZGB_NCH; d++)
        ch[d] = 0.0;
    if (s == 0)
        ch[0] = y;
    for (d = 0; d < 4; d++) {
        int q = lat[or_neighbour(M, site, d)];
        if (s == 0 && q == 0)
            ch[1 + d] = (1.0 - y) / 4.0;
        if ((s == 1 && q == 2) || (s == 2 && q == 1))
            ch[5 + d] = OR_PLANT == 6 ? kr / 2.0 : kr / 4.0;
        if (s == 1 && q == 0)
            ch[9 + d] = D / 4.0;
    }
}

/* Conserved spin exchange (Sec. 2, the diffusion example: Kawasaki dynamics,
 * states 0 empty, 1 particle).  A particle at x hops to an empty nearest
 * neighbour x+e_d with the Arrhenius rate (D/4) exp(-(beta * (J * n))), n =
 * the number of occupied neighbours of x.  The hops use the reaction model's
 * channel slots ch9+d (same order), every other channel is 0.              */
static void or_kaw_channels(const or_model* M, const uint8_t* lat, int site, double ch[OR_ZGB_NCH])
{
    double D = M->p[0], J = M->p[1], beta = M->p[2];
    int n = 0, d;
    for (d = 0; d < OR_ZGB_NCH; d++)
        ch[d] = 0.0;
    if (lat[site] != 1)
        return;
    for (d = 0; d < 4; d++)
        n += lat[or_neighbour(M, site, d)] == (OR_PLANT == 12 ? 0 : 1);
    for (d = 0; d < 4; d++)
        if (lat[or_neighbour(M, site, d)] == 0)
            ch[9 + d] = (D / 4.0) * exp(-(beta * (J * (double)n)));
}

static void or_channels(const or_model* M, const uint8_t* lat, int site, double ch[OR_ZGB_NCH])
{
    if (M->model == OR_MODEL_KAW)
        or_kaw_channels(M, lat, site, ch);
    else
        or_zgb_channels(M, lat, site, ch);
}

static double or_zgb_total(const double ch[OR_ZGB_NCH])
{
    double tot = 0.0;
    int c;
    for (c = 0; c < OR_ZGB_NCH; c++) /* left to right, ch0 first */
        tot = tot + ch[c];
    return tot;
}

/* Total rate of all events owned by site x: sum over omega of c(x,omega). */
double or_site_rate(const or_model* M, const uint8_t* lat, int site)
{
    if (M->model == OR_MODEL_FLIP)
        return or_flip_rate(M, lat, site);
    {
        double ch[OR_ZGB_NCH];
        or_channels(M, lat, site, ch);
        return or_zgb_total(ch);
    }
}

/* Apply the event of site x selected with the residual target tg (the part of
 * V*R that falls inside this site's total rate).  For the reaction model the
 * channel is the first positive one whose rate exceeds the remaining target,
 * scanning ch0..ch12 and subtracting; the last positive channel is the
 * fallback.  Writes the changed sites to changed[] and returns their number. */
static int or_apply_event(const or_model* M, uint8_t* lat, int site, double tg, int changed[2])
{
    if (M->model == OR_MODEL_FLIP) {
        lat[site] = (uint8_t)(1 - lat[site]);
        changed[0] = site;
        return 1;
    } else {
        double ch[OR_ZGB_NCH];
        int c, pick = -1, last = -1, d, y;
        or_channels(M, lat, site, ch);
        for (c = 0; c < OR_ZGB_NCH; c++) {
            if (ch[c] == 0.0)
                continue;
            last = c;
            if (tg < ch[c]) {
                pick = c;
                break;
            }
            tg = tg - ch[c];
        }
        if (pick < 0)
            pick = last;
        if (pick == 0) {
            lat[site] = 1;
            changed[0] = site;
            return 1;
        }
        d = OR_PLANT == 9 ? (pick - 1) / 4 : (pick - 1) % 4;
        y = or_neighbour(M, site, d);
        changed[0] = site;
        changed[1] = y;
        if (pick <= 4) {
            lat[site] = 2;
            lat[y] = 2;
        } else if (pick <= 8) {
            lat[site] = 0;
            lat[y] = 0;
        } else {
            lat[site] = 0;
            lat[y] = 1;
        }
        return 2;
    }
}

/* Host copy of the per-neighbourhood rates, for comparison with the library's
 * table.  Flip: entry [s*(z+1) + n] for state s and n occupied neighbours.
 * ZGB: entry [pattern*14 + c] for the 13 channels then the total, pattern =
 * s + 3 nE + 9 nW + 27 nN + 81 nS.  Computed through the same per-site rate
 * functions on a small scratch lattice, so it restates the definitions above. */
int or_rate_table(const or_model* M, double* out, int n)
{
    if (M->model == OR_MODEL_FLIP) {
        int z = or_ndir(M), s, k;
        if (n < 2 * (z + 1))
            return OR_EINVAL;
        for (s = 0; s < 2; s++)
            for (k = 0; k <= z; k++) {
                if (s == 0)
                    out[s * (z + 1) + k] = M->p[0];
                else
                    out[s * (z + 1) + k] = M->p[1] * exp(-(M->p[4] * (M->p[2] * (double)k + M->p[3])));
            }
        return 2 * (z + 1);
    } else {
        /* a 3x3 periodic scratch lattice: the centre (1,1) has four distinct
         * neighbours E=(2,1), W=(0,1), N=(1,2), S=(1,0)                      */
        or_model T = *M;
        uint8_t lat[9];
        int pat;
        T.dim = 2;
        T.Lx = 3;
        T.Ly = 3;
        if (n < 243 * 14)
            return OR_EINVAL;
        for (pat = 0; pat < 243; pat++) {
            double ch[OR_ZGB_NCH];
            int c, r = pat;
            memset(lat, 0, 9);
            lat[4] = (uint8_t)(r % 3); r /= 3;
            lat[5] = (uint8_t)(r % 3); r /= 3;
            lat[3] = (uint8_t)(r % 3); r /= 3;
            lat[7] = (uint8_t)(r % 3); r /= 3;
            lat[1] = (uint8_t)(r % 3);
            or_channels(&T, lat, 4, ch);
            for (c = 0; c < OR_ZGB_NCH; c++)
                out[pat * 14 + c] = ch[c];
            out[pat * 14 + 13] = or_zgb_total(ch);
        }
        return 243 * 14;
    }
}

/* ------------------------------------------------------------------------ */
/* Sum tree over n leaves (n padded to a power of two with +0.0), heap layout:
 * v[1] is the root, node k has children 2k, 2k+1, leaf i sits at v[nt + i].
 * Internal nodes are always left + right of their current children.          */
static int or_pow2(int n)
{
    int p = 1;
    while (p < n)
        p <<= 1;
    return p;
}

static void or_tree_build(double* v, int nt)
{
    int k;
    for (k = nt - 1; k >= 1; k--)
        v[k] = v[2 * k] + v[2 * k + 1];
}

/* Descent with target tg in [0, root): at node k go left when tg < left or
 * when the right subtree is empty, otherwise subtract left and go right.
 * Returns the leaf index and leaves the residual target in *tg.              */
static int or_tree_descend(const double* v, int nt, double* tg)
{
    int k = 1;
    double t = *tg;
    while (k < nt) {
        double L = v[2 * k], Rr = v[2 * k + 1];
        if (t < L || Rr == 0.0) {
            k = 2 * k;
        } else {
            t = OR_PLANT == 3 ? t - Rr : t - L;
            k = 2 * k + 1;
        }
    }
    *tg = t;
    return k - nt;
}

/* Exposed for the selection tests: build a tree over leaves[0..n) and select
 * with V in [0,1) (target V * root).  Returns -1 when the root is zero.      */
int or_tree_select(const double* leaves, int n, double V, double* root_out, double* resid_out)
{
    int nt = or_pow2(n), i, leaf;
    double* v = (double*)calloc((size_t)(2 * nt), sizeof(double));
    double tg;
    if (!v)
        return OR_ENOMEM;
    for (i = 0; i < n; i++)
        v[nt + i] = leaves[i];
    or_tree_build(v, nt);
    if (root_out)
        *root_out = v[1];
    if (v[1] == 0.0) {
        free(v);
        return -1;
    }
    tg = V * v[1];
    leaf = or_tree_descend(v, nt, &tg);
    if (resid_out)
        *resid_out = tg;
    free(v);
    return leaf;
}

/* ------------------------------------------------------------------------ */
/* Observables: integer counts of sites per state and of nearest-neighbour
 * bonds (each bond once, along +x and, in 2D, +y) whose two ends are both in
 * state k, plus the number of A-B bonds.  out[0..2] = #sites in state 0..2,
 * out[3..5] = #bonds k-k, out[6] = #bonds A-B.                               */
void or_observe(const or_model* M, const uint8_t* lat, int64_t out[7])
{
    int N = M->Lx * M->Ly, i, k;
    for (k = 0; k < 7; k++)
        out[k] = 0;
    for (i = 0; i < N; i++) {
        int s = lat[i], d;
        out[s] += 1;
        for (d = 0; d < or_ndir(M); d += 2) {
            int q = lat[or_neighbour(M, i, d)];
            if (q == s)
                out[3 + s] += 1;
            if ((s == 1 && q == 2) || (s == 2 && q == 1))
                out[6] += 1;
        }
    }
}

/* Bernoulli(p) initial lattice: site i is 1 when V < p, with V from Philox at
 * counter (i, 0, 0, 1) and key (seed, replica).                             */
void or_init_bernoulli(uint8_t* lat, int64_t N, double p, uint32_t seed, uint32_t replica)
{
    int64_t i;
    for (i = 0; i < N; i++) {
        double U, V;
        or_draw((uint32_t)i, 0u, 0u, 1u, seed, replica, &U, &V);
        lat[i] = (uint8_t)(V < p ? 1 : 0);
    }
}

/* ------------------------------------------------------------------------ */
/* (a) Exact serial SSA of the whole lattice (eqs. totalrate, skeleton).
 * Time draws use counter (e_lo, e_hi, 0xFFFFFFFF, 2).  Observables are
 * recorded at the given increasing sample times: the state after the last
 * event with time < t_k.  obs_out holds 7 int64 per sample.                  */
int or_ssa_serial(const or_model* M, uint8_t* lat, double T, uint32_t seed, uint32_t replica,
                  const double* sample_t, int n_samples, int64_t* obs_out, uint64_t* events_out)
{
    int N = M->Lx * M->Ly, nt = or_pow2(N), i, next = 0;
    double* v = (double*)calloc((size_t)(2 * nt), sizeof(double));
    double t = 0.0;
    uint64_t e = 0;
    if (!v)
        return OR_ENOMEM;
    for (i = 0; i < N; i++)
        v[nt + i] = or_site_rate(M, lat, i);
    or_tree_build(v, nt);
    for (;;) {
        double R = v[1], U, V, tn, tg;
        int site, changed[2], nc, c;
        if (R == 0.0)
            break;
        or_draw((uint32_t)e, (uint32_t)(e >> 32), 0xFFFFFFFFu, 2u, seed, replica, &U, &V);
        tn = t + (-or_log(U)) / R;
        while (next < n_samples && sample_t[next] <= tn && sample_t[next] <= T) {
            or_observe(M, lat, obs_out + 7 * next);
            next++;
        }
        if (!(tn < T))
            break;
        t = tn;
        tg = V * R;
        site = or_tree_descend(v, nt, &tg);
        nc = or_apply_event(M, lat, site, tg, changed);
        /* rates of the changed sites and of their neighbours, then ancestors */
        for (c = 0; c < nc; c++) {
            int d;
            for (d = -1; d < or_ndir(M); d++) {
                int s = d < 0 ? changed[c] : or_neighbour(M, changed[c], d);
                int k = nt + s;
                v[k] = or_site_rate(M, lat, s);
                for (k = k / 2; k >= 1; k /= 2)
                    v[k] = v[2 * k] + v[2 * k + 1];
            }
        }
        e++;
    }
    while (next < n_samples) {
        or_observe(M, lat, obs_out + 7 * next);
        next++;
    }
    if (events_out)
        *events_out = e;
    free(v);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Decomposition (Sec. 2.1, eqs. decomposition, sublatt, opdecomp): blocks of
 * bx x by sites tile the lattice; block m = bj*NBX + bi covers
 * x in [bi*bx, (bi+1)*bx), y in [bj*by, (bj+1)*by); colour_map[m] in [0,K).
 * Blocks of one colour must be independent (Sec. 2.1, remark after
 * gendecomp): no block of a colour may write a site another block of the same
 * colour reads or writes.  Flip models write C_m and read C_m + N(C_m);
 * pair models read and write C_m + N(C_m).                                   */
static int or_is_pair_model(const or_model* M) { return M->model == OR_MODEL_ZGB || M->model == OR_MODEL_KAW; }

int or_decomp_check(const or_model* M, int bx, int by, int n_colours, const int* colour_map)
{
    int N = M->Lx * M->Ly, NBX, NBY, nb, m, m2, i;
    char *Rm, *Wm;
    if (bx <= 0 || by <= 0 || M->Lx % bx || M->Ly % by || n_colours <= 0)
        return OR_EINVAL;
    NBX = M->Lx / bx;
    NBY = M->Ly / by;
    nb = NBX * NBY;
    for (m = 0; m < nb; m++)
        if (colour_map[m] < 0 || colour_map[m] >= n_colours)
            return OR_EINVAL;
    Rm = (char*)calloc((size_t)nb * N, 1);
    Wm = (char*)calloc((size_t)nb * N, 1);
    if (!Rm || !Wm) {
        free(Rm);
        free(Wm);
        return OR_ENOMEM;
    }
    for (m = 0; m < nb; m++) {
        int bi = m % NBX, bj = m / NBX, x, y, d;
        for (y = bj * by; y < (bj + 1) * by; y++)
            for (x = bi * bx; x < (bi + 1) * bx; x++) {
                int s = y * M->Lx + x;
                Rm[(size_t)m * N + s] = 1;
                Wm[(size_t)m * N + s] = 1;
                for (d = 0; d < or_ndir(M); d++) {
                    int q = or_neighbour(M, s, d);
                    Rm[(size_t)m * N + q] = 1;
                    if (or_is_pair_model(M))
                        Wm[(size_t)m * N + q] = 1;
                }
            }
    }
    for (m = 0; m < nb; m++)
        for (m2 = m + 1; m2 < nb; m2++) {
            if (colour_map[m] != colour_map[m2])
                continue;
            for (i = 0; i < N; i++) {
                char wa = Wm[(size_t)m * N + i], wb = Wm[(size_t)m2 * N + i];
                char ra = Rm[(size_t)m * N + i], rb = Rm[(size_t)m2 * N + i];
                if ((wa && (rb || wb)) || (wb && ra)) {
                    free(Rm);
                    free(Wm);
                    return OR_EDECOMP;
                }
            }
        }
    free(Rm);
    free(Wm);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Schedules (Sec. 2.2 eq. lie; Sec. 3 eqs. PCSl, strang, PCSs; Sec. 3.1 eq.
 * SLPCS).  One step of length dt is a list of windows (colour, duration):
 *   Lie:    (0,dt), (1,dt), ..., (K-1,dt)
 *   Strang: (0,h), ..., (K-2,h), (K-1,dt), (K-2,h), ..., (0,h) with h=0.5*dt
 *   Random: K windows of length dt, each of a colour drawn uniformly from
 *           Philox at counter (w, 0, 0, 3): colour = floor(V*K).
 * n_steps = T/dt must be an integer to within 1e-9 relative.  step_end[w] is
 * 1 for the last window of each step.  Returns the number of windows.        */
int64_t or_schedule(int split, int n_colours, double dt, double T, uint32_t seed, uint32_t replica,
                    int64_t max_windows, int* colour_out, double* dur_out, uint8_t* step_end_out)
{
    double nd;
    int64_t n_steps, per_step, w = 0, k;
    int c;
    double h = 0.5 * dt;
    if (!(dt > 0.0) || !(T >= 0.0) || n_colours < 1)
        return OR_EINVAL;
    nd = floor(T / dt + 0.5);
    if (fabs(nd * dt - T) > 1e-9 * (T > 1.0 ? T : 1.0))
        return OR_EINVAL;
    n_steps = (int64_t)nd;
    per_step = (split == OR_STRANG) ? (2 * n_colours - 1) : n_colours;
    if (split != OR_LIE && split != OR_STRANG && split != OR_RANDOM)
        return OR_EINVAL;
    if (colour_out == NULL)
        return n_steps * per_step;
    if (n_steps * per_step > max_windows)
        return OR_EINVAL;
    for (k = 0; k < n_steps; k++) {
        for (c = 0; c < per_step; c++) {
            int col;
            double dur;
            if (split == OR_LIE) {
                col = c;
                dur = dt;
            } else if (split == OR_STRANG) {
                col = c < n_colours ? c : 2 * (n_colours - 1) - c;
                dur = (col == n_colours - 1 && OR_PLANT != 4) ? dt : h;
            } else {
                double U, V;
                or_draw((uint32_t)(OR_PLANT == 10 ? k : w), 0u, 0u, 3u, seed, replica, &U, &V);
                col = (int)(V * (double)n_colours);
                dur = dt;
            }
            colour_out[w] = col;
            dur_out[w] = dur;
            if (step_end_out)
                step_end_out[w] = (uint8_t)(c == per_step - 1);
            w++;
        }
    }
    return w;
}

/* ------------------------------------------------------------------------ */
/* (b) One block-window: the serial SSA kernel of block m for duration dur
 * with every site outside the block frozen (Sec. 2.2, Steps 1-3).  Leaves are
 * the block's sites in row-major order.  Draw e of window w uses Philox
 * counter (e, m, w, 0); the draw that overshoots the window is discarded.
 * Returns the number of accepted events.  After each event the whole block
 * tree is rebuilt from the lattice (plain and obviously a pure function of it). */
static uint32_t or_block_window(const or_model* M, uint8_t* lat, int bx, int by, int m, int NBX,
                                double dur, uint64_t w, uint32_t seed, uint32_t replica, double* v)
{
    int n = bx * by, nt = or_pow2(n), i;
    int x0 = (m % NBX) * bx, y0 = (m / NBX) * by;
    double t = 0.0;
    uint32_t e = 0;
    for (;;) {
        double R, U, V, tn, tg;
        int leaf, site, changed[2];
        for (i = 0; i < nt; i++)
            v[nt + i] = 0.0;
        for (i = 0; i < n; i++)
            v[nt + i] = or_site_rate(M, lat, (y0 + i / bx) * M->Lx + x0 + i % bx);
        or_tree_build(v, nt);
        R = v[1];
        if (R == 0.0)
            break;
        or_draw(e, (uint32_t)m, (uint32_t)w, 0u, seed, replica, &U, &V);
        tn = t + (-or_log(U)) / R;
        if (!(tn < dur))
            break;
        t = tn;
        tg = V * R;
        leaf = or_tree_descend(v, nt, &tg);
        site = (y0 + leaf / bx) * M->Lx + x0 + leaf % bx;
        or_apply_event(M, lat, site, tg, changed);
        e++;
    }
    return e;
}

/* Run windows [0, n_windows) of a schedule (colour, duration per window) on
 * the lattice in place.  The Philox window index of local window i is w0 + i.
 * Blocks of the active colour run in block-id order (they are independent, so
 * the order does not change the result).  Optional outputs:
 *   W_out[i*nb + m]     accepted events of block m in window i (0 if inactive)
 *   snap_out[i*N ...]   the lattice after window i
 *   obs_out             7 counts after every window whose observe flag is set
 *   events_out          total accepted events                                */
int or_fs_run(const or_model* M, uint8_t* lat, int bx, int by, int n_colours, const int* colour_map,
              const int* win_colour, const double* win_dur, int64_t n_windows, uint64_t w0,
              uint32_t seed, uint32_t replica, uint32_t* W_out, uint8_t* snap_out,
              const uint8_t* observe_flags, int64_t* obs_out, uint64_t* events_out)
{
    int N = M->Lx * M->Ly, NBX, NBY, nb, m;
    int64_t i, n_obs = 0;
    uint64_t total = 0;
    double* v;
    if (bx <= 0 || by <= 0 || M->Lx % bx || M->Ly % by)
        return OR_EINVAL;
    NBX = M->Lx / bx;
    NBY = M->Ly / by;
    nb = NBX * NBY;
    v = (double*)calloc((size_t)(2 * or_pow2(bx * by)), sizeof(double));
    if (!v)
        return OR_ENOMEM;
    for (i = 0; i < n_windows; i++) {
        int col = win_colour[i];
        for (m = 0; m < nb; m++) {
            uint32_t e = 0;
            if (colour_map[m] == col || OR_PLANT == 7) {
                e = or_block_window(M, lat, bx, by, m, NBX, win_dur[i], w0 + (uint64_t)i, seed, replica, v);
                total += e;
            }
            if (W_out)
                W_out[i * nb + m] = e;
        }
        if (snap_out)
            memcpy(snap_out + i * N, lat, (size_t)N);
        if (observe_flags && observe_flags[i]) {
            or_observe(M, lat, obs_out + 7 * n_obs);
            n_obs++;
        }
    }
    if (events_out)
        *events_out = total;
    free(v);
    (void)n_colours;
    return OR_OK;
}
