// Tiling of the fused three-step Chebyshev block (host side): the one place that decides
// the launch shape of that kernel, so a record of its measured traffic can name it.
#pragma once

#include <algorithm>

#include "ac_internal.h"

namespace ac {

// One tile per workgroup and a wave per shift group (`groups` waves per block).  Strips
// of 64*vx computed columns advance by 64*vx - 4; vx = 2 points per lane in float32 on
// even grids at least 128 wide, else 1 (vx_pref > 0 overrides where allowed).  The
// automatic height aims at about one round of occ * 1024 / groups workgroups (occ waves
// per SIMD on 256 CUs x 4 SIMDs), at least 4 and at most 256 rows; h_pref > 0 sets it.
inline Tiling triple_tiling(const Geom& g, bool fp64, int groups, int h_pref, int vx_pref, int occ) {
    Tiling t{};
    int vx = vx_pref > 0 ? vx_pref : (fp64 ? 1 : 2);
    if (g.nx % 2 != 0 || g.nx < 128) vx = 1;
    t.vx = vx;
    t.wpb = groups;
    const int stride = kWave * vx - 4;
    const int inner = g.nx - 2;  // columns past the first strip's low ghost edge
    t.nsx = (inner + stride - 1) / stride;
    const long long slots = static_cast<long long>(occ) * 1024;
    const long long want = std::max<long long>(1, slots / groups);  // workgroups in one round
    const int h = static_cast<int>((static_cast<long long>(t.nsx) * g.ny + want - 1) / want);
    t.h = h_pref > 0 ? h_pref : std::min(256, std::max(4, h));
    if (t.h > g.ny) t.h = g.ny;
    t.ncy = (g.ny + t.h - 1) / t.h;
    t.tiles = static_cast<long long>(t.nsx) * t.ncy;
    t.blocks = static_cast<int>(t.tiles);
    return t;
}

}  // namespace ac
