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
// boundary rows and columns (written) and their neighbours (read, or written
// for pair events), which is the per-site check's set of marks restricted to
// the sites two blocks can share; the verdict is the same.  Owner marks are
// stamped with the colour instead of being cleared for every colour.
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

// Neighbour of a site in direction d (0 +x, 1 -x, 2 +y, 3 -y), periodic.
inline int64_t decomp_nbr(const DecompGeom& G, int64_t s, int d)
{
    int64_t x = s % G.Lx, y = s / G.Lx;
    switch (d) {
    case 0: x = (x + 1) % G.Lx; break;
    case 1: x = (x + G.Lx - 1) % G.Lx; break;
    case 2: y = (y + 1) % G.Ly; break;
    default: y = (y + G.Ly - 1) % G.Ly; break;
    }
    return y * G.Lx + x;
}

// True when two blocks of one colour interact; then *bad_colour and *bad_site
// name the colour and a site where they meet.  blocks[colour_off[c] ..
// colour_off[c+1]) are the blocks of colour c.
inline bool decomp_conflict(const DecompGeom& G, bool pair, int n_colours, const int32_t* blocks,
                            const int32_t* colour_off, int* bad_colour, int64_t* bad_site)
{
    const int64_t N = G.Lx * G.Ly;
    const int nd = G.dim == 1 ? 2 : 4;
    std::unique_ptr<int32_t[]> ownW(new int32_t[(size_t)N]), ownR(new int32_t[(size_t)N]);
    std::vector<int16_t> stamp((size_t)N, (int16_t)-1); // colour whose marks ownW/ownR hold
    for (int c = 0; c < n_colours; ++c) {
        // mark site s for block m: conflict when another block wrote it, or
        // when m writes it and another block read it
        auto mark = [&](int64_t s, int32_t m, bool write) -> bool {
            if (stamp[(size_t)s] != c) {
                stamp[(size_t)s] = (int16_t)c;
                ownW[(size_t)s] = -1;
                ownR[(size_t)s] = -1;
            }
            int32_t& w = ownW[(size_t)s];
            int32_t& r = ownR[(size_t)s];
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
            const int64_t x0 = (int64_t)(m % G.NBX) * G.bx, y0 = (int64_t)(m / G.NBX) * G.by;
            for (int64_t y = y0; y < y0 + G.by; ++y) {
                const bool edge_row = G.dim == 2 && (y == y0 || y == y0 + G.by - 1);
                // the whole row on the block's top and bottom, else its two ends
                const int64_t step = edge_row || G.bx <= 2 ? 1 : G.bx - 1;
                for (int64_t x = x0; x < x0 + G.bx; x += step) {
                    const int64_t s = y * G.Lx + x;
                    bool ok = mark(s, m, true);
                    for (int d = 0; d < nd && ok; ++d)
                        ok = mark(decomp_nbr(G, s, d), m, pair);
                    if (!ok) {
                        *bad_colour = c;
                        *bad_site = s;
                        return true;
                    }
                }
            }
        }
    }
    return false;
}

} // namespace fskmc
