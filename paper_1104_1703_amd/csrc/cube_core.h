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

// The same pass followed by the residual r = L x - f of the cube's cells and
// its R1 restriction onto the 4 x 4 x 4 coarse cells the cube covers (Sec. 2
// steps 2-4; coarse right-hand side -(1/8) of the sum of the active
// children's residuals, 0 off the coarse domain): the residual needs the
// pass's black values on a 1-cell ring too, so red runs on the cube plus a
// 2-cell ring, black on the cube plus a 1-cell ring, from a 14^3 x region
// (3-cell halo).  Every value is formed with the expression and order of the
// stand-alone pass and restriction, so x and the coarse right-hand side are
// bit for bit theirs.  fc / cd / (cnx, cny, cnz): right-hand side, diagonal
// and dims of the next coarser level.
constexpr int RR = C + 6;                                  // x region with a 3-cell halo
constexpr int RRN = RR * RR * RR;                          // 2744
constexpr int NRED3 = (C + 4) * (C + 4) * (C + 4) / 2;     // red cells on the cube plus a 2-cell ring: 864
constexpr int NBLK3 = (C + 2) * (C + 2) * (C + 2) / 2;     // black cells on the cube plus a 1-cell ring: 500
constexpr int RED_SLOTS = (NRED3 + NT - 1) / NT;           // 4
constexpr int BLK_SLOTS = (NBLK3 + NT - 1) / NT;           // 2

template <typename T>
struct LdsRes {
    T x[RRN];
    T r[C * C * C];
};

template <typename T>
__device__ __forceinline__ void rbgs_cube_restrict(LdsRes<T> &L, const T *__restrict__ xin, T *__restrict__ xout,
                                                   const T *__restrict__ f, const T *__restrict__ d, int nx, int ny,
                                                   int nz, T h2, T ih2, int x0, int y0, int z0,
                                                   const T *__restrict__ cd, T *__restrict__ fc, int cnx, int cny,
                                                   int cnz) {
    const int tid = threadIdx.x;
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
    auto gidx = [&](int gx, int gy, int gz) { return (size_t)gz * sz + (size_t)gy * sy + (size_t)gx; };
    auto inbox = [&](int gx, int gy, int gz) {
        return gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
    };
    constexpr int E = C + 4, EH = E / 2, F = C + 2, FH = F / 2;
    // red cells: region coords in [0, 12), origin two cells before the cube
    // (global i + j + k even: a + b + c even); black: region [0, 10), origin
    // one cell before (global odd: a + b + c even as well, the origin sum is odd)
    int ra[RED_SLOTS], rb[RED_SLOTS], rc[RED_SLOTS], ba[BLK_SLOTS], bb[BLK_SLOTS], bc[BLK_SLOTS];
    T rf[RED_SLOTS], rd[RED_SLOTS], bf[BLK_SLOTS], bd[BLK_SLOTS];
#pragma unroll
    for (int s = 0; s < RED_SLOTS; s++) {
        const int r = tid + s * NT;
        const bool v = r < NRED3;
        const int row = v ? r / EH : 0, m = r % EH;
        rb[s] = row % E;
        rc[s] = row / E;
        ra[s] = ((rb[s] + rc[s]) & 1) + 2 * m;
        const int gx = x0 - 2 + ra[s], gy = y0 - 2 + rb[s], gz = z0 - 2 + rc[s];
        const bool ok = v && inbox(gx, gy, gz);
        rd[s] = ok ? d[gidx(gx, gy, gz)] : T(0);
        rf[s] = ok ? f[gidx(gx, gy, gz)] : T(0);
    }
#pragma unroll
    for (int s = 0; s < BLK_SLOTS; s++) {
        const int r = tid + s * NT;
        const bool v = r < NBLK3;
        const int row = v ? r / FH : 0, m = r % FH;
        bb[s] = row % F;
        bc[s] = row / F;
        ba[s] = ((bb[s] + bc[s]) & 1) + 2 * m;
        const int gx = x0 - 1 + ba[s], gy = y0 - 1 + bb[s], gz = z0 - 1 + bc[s];
        const bool ok = v && inbox(gx, gy, gz);
        bd[s] = ok ? d[gidx(gx, gy, gz)] : T(0);
        bf[s] = ok ? f[gidx(gx, gy, gz)] : T(0);
    }
    // the residual's cells: this thread's two cube cells
    T qf[2], qd[2];
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const int e = tid + s * NT;
        const int a = e % C, b = (e / C) % C, c = e / (C * C);
        const int gx = x0 + a, gy = y0 + b, gz = z0 + c;
        const bool ok = inbox(gx, gy, gz);
        qd[s] = ok ? d[gidx(gx, gy, gz)] : T(0);
        qf[s] = ok ? f[gidx(gx, gy, gz)] : T(0);
    }
    constexpr int XL = (RRN + NT - 1) / NT;  // 11
    T xv[XL];
#pragma unroll
    for (int q = 0; q < XL; q++) {
        const int e = tid + q * NT;
        const int u = e % RR, v = (e / RR) % RR, w = e / (RR * RR);
        const int gx = x0 - 3 + u, gy = y0 - 3 + v, gz = z0 - 3 + w;
        xv[q] = (e < RRN && xin && inbox(gx, gy, gz)) ? xin[gidx(gx, gy, gz)] : T(0);
    }
#pragma unroll
    for (int q = 0; q < XL; q++) {
        const int e = tid + q * NT;
        if (e < RRN) L.x[e] = xv[q];
    }
    __syncthreads();
    auto nbs = [&](int q) {
        const T *c = L.x;
        return (c[q - 1] + c[q + 1]) + (c[q - RR] + c[q + RR]) + (c[q - RR * RR] + c[q + RR * RR]);
    };
    auto relax = [&](int q, T fv, T dv) {
        const T s = nbs(q);
        L.x[q] = (s - h2 * fv) / dv;
    };
#pragma unroll
    for (int s = 0; s < RED_SLOTS; s++)
        if (rd[s] != T(0)) relax(((rc[s] + 1) * RR + (rb[s] + 1)) * RR + (ra[s] + 1), rf[s], rd[s]);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < BLK_SLOTS; s++)
        if (bd[s] != T(0)) relax(((bc[s] + 2) * RR + (bb[s] + 2)) * RR + (ba[s] + 2), bf[s], bd[s]);
    __syncthreads();
    // store the cube and form its residual
#pragma unroll
    for (int s = 0; s < 2; s++) {
        const int e = tid + s * NT;
        const int a = e % C, b = (e / C) % C, c = e / (C * C);
        const int q = ((c + 3) * RR + (b + 3)) * RR + (a + 3);
        const int gx = x0 + a, gy = y0 + b, gz = z0 + c;
        const T xq = L.x[q];
        if (inbox(gx, gy, gz)) xout[gidx(gx, gy, gz)] = xq;
        const T sn = nbs(q);
        L.r[e] = qd[s] != T(0) ? (sn - qd[s] * xq) * ih2 - qf[s] : T(0);
    }
    __syncthreads();
    if (tid < 64) {
        const int I = tid % 4, J = (tid / 4) % 4, K = tid / 16;
        const int gI = x0 / 2 + I, gJ = y0 / 2 + J, gK = z0 / 2 + K;
        if (gI < cnx && gJ < cny && gK < cnz) {
            const size_t P = (size_t)gK * cnx * cny + (size_t)gJ * cnx + gI;
            const T cdv = cd[P];
            T s = T(0);
#pragma unroll
            for (int c = 0; c < 8; c++)  // children in x, y, z order
                s += L.r[((2 * K + (c >> 2)) * C + (2 * J + ((c >> 1) & 1))) * C + (2 * I + (c & 1))];
            fc[P] = cdv != T(0) ? -s / T(8) : T(0);
        }
    }
}

}  // namespace cube
}  // namespace mg
