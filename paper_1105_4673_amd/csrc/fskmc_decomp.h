// Independence of the blocks of each colour (Sec. 2.1, remark after eq.
// gendecomp): no block may write a site that another block of the same colour
// reads or writes.  Spin flip: W = C_m, R = C_m + N(C_m); pair events:
// W = R = C_m + N(C_m).  No HIP dependency, so the check is also compiled and
// tested on its own on the CPU against a per-site check of every site.
//
// Only a block's boundary sites can meet another block: a site whose
// neighbours all lie in its own block is marked by that block alone, and so
// are its neighbours, unless they lie on the boundary, where they are marked
// (as written) when the boundary itself is visited.  So each block marks its
// boundary rows and columns (written) and their neighbours in other blocks
// (read, or written for pair events), which lie on those blocks' boundaries:
// the per-site check's set of marks restricted to the sites two blocks can
// share, so the verdict is the same.  Owner marks are kept per boundary
// position only and stamped with the colour instead of being cleared for
// every colour.
#pragma once
#include <cstdint>
#include <memory>
#include <vector>

namespace fskmc {

// dim 1 or 2 (Ly = 1 in 1D); blocks bx x by tile Lx x Ly, block m = bj * NBX + bi.
struct DecompGeom {
    int dim;
    int64_t Lx, Ly;
    int bx, by, NBX;
};

// True when two blocks of one colour interact; then *bad_colour and *bad_site
// name the colour and a site where they meet.  blocks[colour_off[c] ..
// colour_off[c+1]) are the blocks of colour c.
inline bool decomp_conflict(const DecompGeom& G, bool pair, int n_colours, const int32_t* blocks,
                            const int32_t* colour_off, int* bad_colour, int64_t* bad_site)
{
    const int64_t nb = (G.Lx / G.bx) * (G.Ly / G.by);
    // boundary positions of a block, row by row: a row is visited whole when it
    // is the block's top or bottom row (2D) or the block is at most 2 wide,
    // else at its two ends; pos0[ly] = the first position of row ly
    std::vector<int32_t> pos0((size_t)G.by + 1, 0);
    std::vector<uint8_t> whole((size_t)G.by);
    for (int ly = 0; ly < G.by; ++ly) {
        whole[ly] = (G.dim == 2 && (ly == 0 || ly == G.by - 1)) || G.bx <= 2;
        pos0[ly + 1] = pos0[ly] + (whole[ly] ? G.bx : 2);
    }
    const int64_t R = pos0[G.by];
    const int64_t NBY = G.Ly / G.by;
    // boundary position of site (lx, ly) of block m (the site is on the boundary)
    auto pos = [&](int64_t m, int lx, int ly) -> size_t {
        return (size_t)(m * R + pos0[ly] + (whole[ly] ? lx : (lx ? 1 : 0)));
    };
    // owner marks per boundary position, stamped with the colour they hold
    const size_t M = (size_t)(nb * R);
    std::unique_ptr<int32_t[]> ownW(new int32_t[M]), ownR(new int32_t[M]);
    std::vector<int16_t> stamp(M, (int16_t)-1);
    for (int c = 0; c < n_colours; ++c) {
        // mark boundary position i for block m: conflict when another block
        // wrote it, or when m writes it and another block read it
        auto mark = [&](size_t i, int32_t m, bool write) -> bool {
            if (stamp[i] != c) {
                stamp[i] = (int16_t)c;
                ownW[i] = -1;
                ownR[i] = -1;
            }
            int32_t& w = ownW[i];
            int32_t& r = ownR[i];
            if (write) {
                if ((w != -1 && w != m) || (r != -1 && r != m))
                    return false;
                w = m;
            }
            if (w != -1 && w != m)
                return false;
            if (r == -1)
                r = m;
            else if (r != m)
                r = -2; // several readers: any other writer conflicts
            return true;
        };
        for (int k = colour_off[c]; k < colour_off[c + 1]; ++k) {
            const int32_t m = blocks[k];
            const int64_t bi = m % G.NBX, bj = m / G.NBX;
            // the blocks across each side (periodic; the block itself when it
            // spans the lattice in that direction)
            const int64_t mE = bj * G.NBX + (bi + 1) % G.NBX, mW = bj * G.NBX + (bi + G.NBX - 1) % G.NBX;
            const int64_t mN = ((bj + 1) % NBY) * G.NBX + bi, mS = ((bj + NBY - 1) % NBY) * G.NBX + bi;
            for (int ly = 0; ly < G.by; ++ly) {
                const int step = whole[ly] ? 1 : G.bx - 1;
                for (int lx = 0; lx < G.bx; lx += step) {
                    bool ok = mark(pos(m, lx, ly), m, true);
                    // a neighbour inside the block is the block's own site:
                    // written by it when on its boundary, shared with no other
                    // block otherwise; one across a side lies on the boundary
                    // of the block there
                    if (ok && lx + 1 == G.bx && mE != m)
                        ok = mark(pos(mE, 0, ly), m, pair);
                    if (ok && lx == 0 && mW != m)
                        ok = mark(pos(mW, G.bx - 1, ly), m, pair);
                    if (G.dim == 2) {
                        if (ok && ly + 1 == G.by && mN != m)
                            ok = mark(pos(mN, lx, 0), m, pair);
                        if (ok && ly == 0 && mS != m)
                            ok = mark(pos(mS, lx, G.by - 1), m, pair);
                    }
                    if (!ok) {
                        *bad_colour = c;
                        *bad_site = (bj * G.by + ly) * G.Lx + bi * G.bx + lx;
                        return true;
                    }
                }
            }
        }
    }
    return false;
}

} // namespace fskmc
