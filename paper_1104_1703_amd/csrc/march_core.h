// Residual march of the finest level (device code shared by the per-level
// kernels of transfer.hip and the batched phase kernels of batch.hip).
#pragma once

#include "masked.h"
#include "smooth_core.h"
#include "transfer_core.h"

namespace mg {
namespace tr {

// Residual of the finest level as a march: one block per smoother work item
// (a TX x TY column of cells over a z range of tile pairs), thread (u, v) of
// the tile cross-section owning one cell per plane.  Planes of x pass through
// a 4-plane LDS ring with a 1-cell halo (each loaded once per item); f and
// the code of the thread's own cell stay in registers.  Loads are masked by
// the item's activity masks (granules without active cells read as zero).
// Modes:
//  RM_RESTRICT  R1 restriction: each cell's residual is summed with its x and y
//               partners by lane exchanges (the two rows of a wave are the two
//               y children), and planes 2K and 2K+1 complete coarse plane K:
//               f_c = -(1/8) sum of the 8 children's residuals on active coarse
//               cells, 0 on inactive ones.  Only coarse cells above active
//               finest tiles are written.
//  RM_NORM      sum of r^2 over the item's active cells into part[item] (x may
//               be null: x = 0, r = -f).
//  RM_NORM32    as RM_NORM, and -r is written in float to r32 on active cells.
//  RM_AXPY32    the correction is added first: the residual and norm are those
//               of x + e (e a float correction), x + e is written to xo on
//               active cells (xo != x: neighbouring items read x as halo) and
//               -r in float to r32.
enum { RM_RESTRICT = 0, RM_NORM = 1, RM_NORM32 = 2, RM_AXPY32 = 3 };
namespace rm {
constexpr int PX = TX + 2, PY = TY + 2, PN = PX * PY;  // x plane, 1-cell halo
constexpr int XR = (PN + NT - 1) / NT;
constexpr int PF = 4;
constexpr int XS = 4;
}  // namespace rm

// One work item of the residual march (called by all NT threads of a block);
// pm: the item's SEGZ + 4 activity masks.  Returns the thread's sum of r^2
// (the norm modes; the caller reduces it).
template <typename T>
struct ResLds {
    T xs[rm::XS][rm::PN];
    unsigned long long ms[rb::MAXPL];
};

template <typename T, int SEGZ, int MODE>
__device__ __forceinline__ double residual_item(ResLds<T> &L, const T *__restrict__ x, const T *__restrict__ f,
                                                const uint8_t *__restrict__ code, int nx, int ny, int nz, T ih2,
                                                const Seg sg, const unsigned long long *__restrict__ pm,
                                                const T *__restrict__ cd, int cnx, int cny, T *__restrict__ fc,
                                                float *__restrict__ r32, const float *__restrict__ ecor,
                                                T *__restrict__ xo) {
    using namespace rm;
    static_assert(SEGZ + 4 <= rb::MAXPL, "work item longer than the mask array");
    auto &xs = L.xs;
    auto &ms = L.ms;
    const int tid = threadIdx.x;
    if (tid < SEGZ + 4) ms[tid] = pm[tid];
    const int gx0 = sg.x0 - 1, gy0 = sg.y0 - 1;
    const int z0 = max(sg.z0, 0), z1 = min(sg.z1, nz);
    const size_t plane = (size_t)nx * ny;
    const int pbytes = (int)(plane * sizeof(T));
    constexpr int TSH = sizeof(T) == 8 ? 3 : 2;  // byte offset -> element offset
    // plane elements of this thread (x with halo) and its own cell: byte
    // offsets (OFF_NONE outside the box) and mask bits (one byte each)
    int xoff[XR];
    unsigned bits = 0;
#pragma unroll
    for (int q = 0; q < XR; q++) {
        const int e = min(tid + q * NT, PN - 1);
        const int gx = gx0 + e % PX, gy = gy0 + e / PX;
        const bool in = (tid + q * NT < PN) && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        xoff[q] = in ? (gy * nx + gx) * (int)sizeof(T) : OFF_NONE;
        bits |= (unsigned)item_mask_bit(e % PX + 1, e / PX + 1) << (8 * q);
    }
    static_assert(XR < 4, "mask bit indices are packed into one word");
    const int u = tid % TX, v = tid / TX;
    const int ci = sg.x0 + u, cj = sg.y0 + v;
    const bool own = ci < nx && cj < ny;
    const int coff = own ? (cj * nx + ci) * (int)sizeof(T) : OFF_NONE;
    bits |= (unsigned)item_mask_bit(u + 2, v + 2) << (8 * XR);
    const int q0 = (v + 1) * PX + (u + 1);  // own cell in the x plane
    __syncthreads();  // masks
    auto mbit = [&](unsigned long long m, int j) { return (bool)((m >> ((bits >> (8 * j)) & 63u)) & 1ull); };

    struct Regs {
        T x[XR];
        float e[MODE == RM_AXPY32 ? XR : 1];
        T f;
        uint8_t c;
    };
    // plane k = z0 - 2 + pi
    auto fetch = [&](Regs &r, int k, int pi) {
        const unsigned long long m = (k >= 0 && k < nz) ? ms[pi] : 0ull;
        const size_t base = (size_t)min(max(k, 0), nz - 1) * plane;
        const __amdgpu_buffer_rsrc_t rx = rsrc(x ? x + base : f + base, x ? pbytes : 0);
#pragma unroll
        for (int q = 0; q < XR; q++) r.x[q] = bload<T>(rx, mbit(m, q) ? xoff[q] : OFF_NONE);
        if constexpr (MODE == RM_AXPY32) {
            const __amdgpu_buffer_rsrc_t re = rsrc(ecor + base, (int)(plane * sizeof(float)));
#pragma unroll
            for (int q = 0; q < XR; q++)
                r.e[q] = bload<float>(re, mbit(m, q) && xoff[q] != OFF_NONE ? xoff[q] >> (TSH - 2) : OFF_NONE);
        }
        const int oo = mbit(m, XR) ? coff : OFF_NONE;
        r.f = bload<T>(rsrc(f + base, pbytes), oo);
        r.c = bload<uint8_t>(rsrc(code + base, (int)plane), oo == OFF_NONE ? OFF_NONE : oo >> TSH);
    };
    auto commit = [&](const Regs &r, int j) {  // plane z0 + j, j >= -1
        T *d = xs[(j + XS) % XS];
#pragma unroll
        for (int q = 0; q < XR; q++) {
            if (tid + q * NT >= PN) continue;
            if constexpr (MODE == RM_AXPY32) d[tid + q * NT] = r.x[q] + (T)r.e[q];
            else d[tid + q * NT] = r.x[q];
        }
    };

    // steps commit planes z0-1 .. z0+SEGZ; the step of plane p computes the
    // residual of plane p-1 (f and code of plane p-1 held from the previous step)
    constexpr int NSTEP = SEGZ + 2;
    Regs r[PF];
#pragma unroll
    for (int q = 0; q < PF; q++) fetch(r[q], z0 - 1 + q, q + 1);
    T hold_f = T(0), acc = T(0);
    double sq = 0.0;
    uint8_t hold_c = CODE_OFF;
#pragma unroll
    for (int st = 0; st < NSTEP; st++) {
        const int j = st - 2;  // plane z0 + j gets its residual in this step
        const T fprev = hold_f;
        const uint8_t cprev = hold_c;
        hold_f = r[st % PF].f;
        hold_c = r[st % PF].c;
        commit(r[st % PF], j + 1);
        if (st + PF < NSTEP) fetch(r[st % PF], z0 + j + 1 + PF, st + 1 + PF);
        __syncthreads();
        const int k = z0 + j;
        if (j >= 0 && k < z1) {  // uniform
            const T *xc = xs[(j + XS) % XS];
            const T *xd = xs[(j - 1 + XS) % XS];
            const T *xu = xs[(j + 1 + XS) % XS];
            T rr = T(0);
            if (cprev != CODE_OFF) {
                const T d = T((int)cprev);
                const T sum = ((xc[q0 - 1] + xc[q0 + 1]) + (xc[q0 - PX] + xc[q0 + PX])) + (xd[q0] + xu[q0]);
                rr = (sum - d * xc[q0]) * ih2 - fprev;
            }
            if constexpr (MODE == RM_RESTRICT) {
                T s2 = rr + __shfl_xor(rr, 1);
                s2 += __shfl_xor(s2, 32);
                if ((k & 1) == 0) {
                    acc = s2;
                } else {
                    acc += s2;
                    if ((u & 1) == 0 && (v & 1) == 0 && own) {
                        const size_t P = ((size_t)(k >> 1) * cny + (cj >> 1)) * cnx + (ci >> 1);
                        fc[P] = cd[P] != T(0) ? -acc / T(8) : T(0);
                    }
                }
            } else {
                sq += (double)rr * (double)rr;
                const bool act = cprev != CODE_OFF;
                if constexpr (MODE == RM_NORM32 || MODE == RM_AXPY32)
                    bstore<float>((float)(-rr), rsrc(r32 + (size_t)k * plane, (int)(plane * sizeof(float))),
                                  act ? coff >> (TSH - 2) : OFF_NONE);
                if constexpr (MODE == RM_AXPY32)
                    bstore<T>(xc[q0], rsrc(xo + (size_t)k * plane, pbytes), act ? coff : OFF_NONE);
            }
        }
    }
    return sq;
}

}  // namespace tr
}  // namespace mg
