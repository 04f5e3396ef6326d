// Tile geometry shared by every stencil kernel of the library: work is
// issued over TX x TY x TZ blocks of a level's (nz, ny, nx) box.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace mg {

constexpr int TX = 32;  // tile width along x (one 256-byte row of doubles)
constexpr int TY = 8;
constexpr int TZ = 8;
constexpr int SEG_TILES_FINE = 2;    // default z-tiles per smoother work item on the finest level
constexpr int SEGZ_COARSE1 = 4;      // default planes per smoother work item on level 1
constexpr int SEGZ_COARSE = 2;       // default planes per smoother work item on coarser levels (latency-bound: short marches)
constexpr int SEGZ_FINE_MAX = 32;    // longest finest-level work item with kernel instances (8, 16, 32 planes)
// Finest-level cell code: the diagonal of the cell's equation, 12 - (number
// of active face neighbours) = 6..12 for an active cell, CODE_OFF if inactive.
constexpr uint8_t CODE_OFF = 0;

// Smoother work item: origin of an xy tile and a z range [z0, z1).
struct Seg {
    int x0, y0, z0, z1;
};

}  // namespace mg
