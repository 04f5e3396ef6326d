// Masked global memory access for the finest-level kernels that march over
// the smoother's work items.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tiles.h"

namespace mg {

// Activity mask of a work item (a TX x TY column of cells at (x0, y0) over
// planes [z0, z1) of at most SEGZ planes): one word for each of its planes
// z0-2 .. z0+SEGZ+1, in which bit 4 v + g is set when row y = y0-2+v
// (0 <= v < TY+4) holds an active cell in granule g of the row, the granules
// being x0-2..x0-1, x0..x0+15, x0+16..x0+31 and x0+32..x0+33 (each inside one
// 128-byte line of doubles).  Words of planes outside the box or above z1+1
// are zero.  Loads of a granule without active cells are skipped: inactive
// cells hold x = 0 in every iterate buffer and their f and diagonal are never
// used.  (u, v): cell (x0-2+u, y0-2+v).
__host__ __device__ constexpr int item_mask_bit(int u, int v) { return 4 * v + ((u + 14) >> 4); }

// Buffer-resource access: a lane whose byte offset lies beyond the resource
// size reads 0 and writes nothing without touching memory, so a masked lane
// costs no traffic while every lane issues the same instructions (exact wait
// counts in the unrolled march).
constexpr int OFF_NONE = (int)0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
}
template <typename V>
__device__ __forceinline__ V bload(__amdgpu_buffer_rsrc_t r, int off) {
    if constexpr (sizeof(V) == 8) return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else if constexpr (sizeof(V) == 4) return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
    else return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0));
}
template <typename V>
__device__ __forceinline__ void bstore(V v, __amdgpu_buffer_rsrc_t r, int off) {
    using U2 = unsigned __attribute__((ext_vector_type(2)));
    if constexpr (sizeof(V) == 8) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, off, 0, 0);
    else __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}

}  // namespace mg
