// The library's block-independence check (fskmc_decomp.h), which marks only
// block boundaries, against a check that marks every site of every block and
// its neighbours, written here on its own: the same verdict on every
// configuration of a sweep over lattice and block shapes (1D and 2D, one and
// two blocks across a periodic direction), built-in 2- and 4-colour maps and
// random colour maps, spin flip and pair events.
#include "../../paper_1105_4673_amd/csrc/fskmc_decomp.h"

#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

using fskmc::DecompGeom;

// neighbour of a site in direction d (0 +x, 1 -x, 2 +y, 3 -y), periodic
static int64_t site_nbr(const DecompGeom& G, int64_t s, int d)
{
    int64_t x = s % G.Lx, y = s / G.Lx;
    if (d == 0)
        x = (x + 1) % G.Lx;
    else if (d == 1)
        x = (x + G.Lx - 1) % G.Lx;
    else if (d == 2)
        y = (y + 1) % G.Ly;
    else
        y = (y + G.Ly - 1) % G.Ly;
    return y * G.Lx + x;
}

// every site of every block of a colour: own sites written, neighbours read
// (written for pair events); a conflict is a site written by one block and
// touched by another
static bool conflict_all_sites(const DecompGeom& G, bool pair, int K, const std::vector<int>& cmap)
{
    const int64_t N = G.Lx * G.Ly;
    const int nd = G.dim == 1 ? 2 : 4;
    const int nb = (int)cmap.size();
    for (int c = 0; c < K; ++c) {
        std::vector<std::vector<int>> writers((size_t)N), touchers((size_t)N);
        for (int m = 0; m < nb; ++m) {
            if (cmap[m] != c)
                continue;
            const int64_t x0 = (int64_t)(m % G.NBX) * G.bx, y0 = (int64_t)(m / G.NBX) * G.by;
            for (int64_t y = y0; y < y0 + G.by; ++y)
                for (int64_t x = x0; x < x0 + G.bx; ++x) {
                    const int64_t s = y * G.Lx + x;
                    writers[s].push_back(m);
                    touchers[s].push_back(m);
                    for (int d = 0; d < nd; ++d) {
                        const int64_t t = site_nbr(G, s, d);
                        touchers[t].push_back(m);
                        if (pair)
                            writers[t].push_back(m);
                    }
                }
        }
        for (int64_t s = 0; s < N; ++s)
            for (int w : writers[s])
                for (int t : touchers[s])
                    if (t != w)
                        return true;
    }
    return false;
}

int main()
{
    std::mt19937 rng(12345);
    long cases = 0, conflicts = 0;
    for (int dim = 1; dim <= 2; ++dim)
        for (int bx = 1; bx <= 5; ++bx)
            for (int by = 1; by <= (dim == 2 ? 4 : 1); ++by)
                for (int NBX = 1; NBX <= 6; ++NBX)
                    for (int NBY = 1; NBY <= (dim == 2 ? 6 : 1); ++NBY)
                        for (int pair = 0; pair <= 1; ++pair)
                            for (int variant = 0; variant < 6; ++variant) {
                                DecompGeom G{dim, (int64_t)bx * NBX, (int64_t)by * NBY, bx, by, NBX};
                                const int nb = NBX * NBY;
                                int K;
                                std::vector<int> cmap(nb);
                                if (variant == 0 || variant == 1) { // built-in checkerboards
                                    K = variant == 0 ? 2 : 4;
                                    for (int m = 0; m < nb; ++m) {
                                        const int bi = m % NBX, bj = m / NBX;
                                        cmap[m] = K == 2 ? (bi + bj) % 2 : (bi % 2) + 2 * (bj % 2);
                                    }
                                } else { // random maps of 1..5 colours
                                    K = 1 + (int)(rng() % 5);
                                    for (int m = 0; m < nb; ++m)
                                        cmap[m] = (int)(rng() % K);
                                }
                                std::vector<int32_t> blocks, off(K + 1, 0);
                                for (int c = 0; c < K; ++c) {
                                    off[c] = (int32_t)blocks.size();
                                    for (int m = 0; m < nb; ++m)
                                        if (cmap[m] == c)
                                            blocks.push_back(m);
                                }
                                off[K] = (int32_t)blocks.size();
                                int bc = -1;
                                int64_t bs = -1;
                                const bool fast = fskmc::decomp_conflict(G, pair, K, blocks.data(), off.data(), &bc, &bs);
                                const bool ref = conflict_all_sites(G, pair, K, cmap);
                                ++cases;
                                conflicts += ref;
                                if (fast != ref) {
                                    std::printf("MISMATCH dim %d block %dx%d grid %dx%d pair %d K %d: boundary %d, "
                                                "all sites %d\n",
                                                dim, bx, by, NBX, NBY, pair, K, (int)fast, (int)ref);
                                    return 1;
                                }
                                if (fast && (bc < 0 || bc >= K || bs < 0 || bs >= G.Lx * G.Ly)) {
                                    std::printf("bad conflict report: colour %d site %lld\n", bc, (long long)bs);
                                    return 1;
                                }
                            }
    std::printf("decomposition ok: %ld cases, %ld with interacting blocks\n", cases, conflicts);
    return 0;
}
