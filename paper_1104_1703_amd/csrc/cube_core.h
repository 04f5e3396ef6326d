// One red-black pass over one 8 x 8 x 8 cube of a coarse level, loaded whole
// (no z march): the alternative work item of the coarse levels, whose passes
// are bound by latency rather than bytes.
#pragma once

#include <hip/hip_runtime.h>

#include "tiles.h"

namespace mg {
namespace cube {

constexpr int C = 8;          // cube edge
constexpr int R = C + 4;      // x region with a 2-cell halo
constexpr int RN = R * R * R; // 1728
constexpr int NT = 256;
constexpr int NRED = (C + 2) * (C + 2) * (C + 2) / 2;  // red cells of the cube plus a 1-cell ring: 500
constexpr int NBLK = C * C * C / 2;                     // black cells of the cube: 256

template <typename T>
struct Lds {
    T x[RN];
};

// The pass the z march gives a coarse tile (Sec. 2 red-black ordering;
// ghost-modified diagonal d): red cells of the cube and of the 1-cell ring
// around it (recomputed by neighbouring cubes from the same inputs), then
// black cells of the cube, each from the same neighbour sum, in the same
// order and the same expression as the march, so the result is bit for bit
// the march's (and the global red-then-black sweep's).  (x0, y0, z0): cube
// origin, multiples of 8.  xin == nullptr: the pass starts from zero.  Every
// in-box cube cell is stored (inactive ones hold their zero).
template <typename T>
__device__ __forceinline__ void rbgs_cube(Lds<T> &L, const T *__restrict__ xin, T *__restrict__ xout,
                                          const T *__restrict__ f, const T *__restrict__ d, int nx, int ny, int nz,
                                          T h2, int x0, int y0, int z0) {
    const int tid = threadIdx.x;
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
    auto gidx = [&](int gx, int gy, int gz) { return (size_t)gz * sz + (size_t)gy * sy + (size_t)gx; };
    auto inbox = [&](int gx, int gy, int gz) {
        return gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
    };
    // this thread's red cells (region coords a, b, c in [0, 10), origin one
    // cell before the cube) and its black cell (cube coords in [0, 8))
    int ra[2], rb[2], rc[2];
    bool rv[2];
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const int r = tid + s * NT;
        rv[s] = r < NRED;
        const int row = rv[s] ? r / 5 : 0, m = r % 5;
        rb[s] = row % (C + 2);
        rc[s] = row / (C + 2);
        ra[s] = ((rb[s] + rc[s] + 1) & 1) + 2 * m;  // red: global i + j + k even
    }
    const int brow = tid / 4, bm = tid % 4;
    const int bb = brow % C, bc = brow / C, ba = ((bb + bc + 1) & 1) + 2 * bm;  // black: odd
    // issue every load: the x region, then f and d of the thread's cells
    T xv[(RN + NT - 1) / NT];
#pragma unroll
    for (int q = 0; q < (RN + NT - 1) / NT; q++) {
        const int e = tid + q * NT;
        const int u = e % R, v = (e / R) % R, w = e / (R * R);
        const int gx = x0 - 2 + u, gy = y0 - 2 + v, gz = z0 - 2 + w;
        xv[q] = (e < RN && xin && inbox(gx, gy, gz)) ? xin[gidx(gx, gy, gz)] : T(0);
    }
    T rf[2], rd[2];
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const int gx = x0 - 1 + ra[s], gy = y0 - 1 + rb[s], gz = z0 - 1 + rc[s];
        const bool ok = rv[s] && inbox(gx, gy, gz);
        rd[s] = ok ? d[gidx(gx, gy, gz)] : T(0);
        rf[s] = ok ? f[gidx(gx, gy, gz)] : T(0);
    }
    T bf = T(0), bd = T(0);
    {
        const int gx = x0 + ba, gy = y0 + bb, gz = z0 + bc;
        if (inbox(gx, gy, gz)) {
            bd = d[gidx(gx, gy, gz)];
            bf = f[gidx(gx, gy, gz)];
        }
    }
#pragma unroll
    for (int q = 0; q < (RN + NT - 1) / NT; q++) {
        const int e = tid + q * NT;
        if (e < RN) L.x[e] = xv[q];
    }
    __syncthreads();
    auto relax = [&](int q, T fv, T dv) {
        const T *c = L.x;
        const T s = (c[q - 1] + c[q + 1]) + (c[q - R] + c[q + R]) + (c[q - R * R] + c[q + R * R]);
        L.x[q] = (s - h2 * fv) / dv;
    };
#pragma unroll
    for (int s = 0; s < 2; s++)
        if (rv[s] && rd[s] != T(0)) relax(((rc[s] + 1) * R + (rb[s] + 1)) * R + (ra[s] + 1), rf[s], rd[s]);
    __syncthreads();
    if (bd != T(0)) relax(((bc + 2) * R + (bb + 2)) * R + (ba + 2), bf, bd);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const int e = tid + s * NT;  // cube cell
        const int a = e % C, b = (e / C) % C, c = e / (C * C);
        const int gx = x0 + a, gy = y0 + b, gz = z0 + c;
        if (inbox(gx, gy, gz)) xout[gidx(gx, gy, gz)] = L.x[((c + 2) * R + (b + 2)) * R + (a + 2)];
    }
}

}  // namespace cube
}  // namespace mg
