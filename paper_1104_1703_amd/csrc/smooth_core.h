// Core of the red-black smoother, shared by the per-level kernels
// (smooth.hip) and the batched persistent kernel (batch.hip).
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include "tiles.h"

namespace mg {
namespace rb {


constexpr int BX = TX, BY = TY;
constexpr int PX = BX + 4, PY = BY + 4, PN = PX * PY;  // x plane with 2-cell halo
constexpr int QX = BX + 2, QY = BY + 2, QN = QX * QY;  // f / diag plane with 1-cell halo
constexpr int NT = 256;
constexpr int XR = (PN + NT - 1) / NT;  // x elements per thread per plane
constexpr int QR = (QN + NT - 1) / NT;  // f elements per thread per plane
constexpr int PF = 4;                   // planes of global loads in flight

// Work items are dealt to the 8 XCDs round-robin by block id; give each XCD a
// contiguous range of work items so that halo re-reads hit its own L2.
__device__ __forceinline__ int xcd_item(int b, int nb) {
    const int per = nb >> 3;  // nb is a multiple of 8
    return (b & 7) * per + (b >> 3);
}

template <typename T, bool FINE>
struct PlaneRegs {
    T x[XR];
    T f[QR];
    typename std::conditional<FINE, uint8_t, T>::type d[QR];  // raw code byte or diagonal
    unsigned ok;  // validity bits: x elements in bits 0..XR-1, f/d elements above
};

// LDS of one work item: a 4-plane ring of x (2-cell halo), and 3-plane rings
// of f and the diagonal (1-cell halo; the finest level keeps its 1-byte
// neighbour code instead of a diagonal).
template <typename T, bool FINE>
struct RbgsLds {
    using DT = typename std::conditional<FINE, uint8_t, T>::type;
    T x[4][PN];
    T f[3][QN];
    DT d[3][QN];
};

// One full red-black pass over one work item (see the file comment of
// smooth.hip).  Called by all 256 threads of a block.
template <typename T, bool FINE, int SEGZ>
__device__ __forceinline__ void rbgs_item(RbgsLds<T, FINE> &L, const T *__restrict__ xin, T *__restrict__ xout,
                                          const T *__restrict__ f, const uint8_t *__restrict__ code,
                                          const T *__restrict__ dco, int nx, int ny, int nz, T h2, const Seg sg) {
    using DT = typename RbgsLds<T, FINE>::DT;
    auto &sx = L.x;
    auto &sf = L.f;
    auto &sd = L.d;
    const int gx0 = sg.x0 - 2, gy0 = sg.y0 - 2;  // origin of the x plane (2-cell halo)
    const size_t plane = (size_t)nx * ny;
    const int tid = threadIdx.x;
    const int z0 = max(sg.z0, 0), z1 = min(sg.z1, nz);  // a work item never leaves the box

    // Per-thread element positions are the same for every plane: precompute
    // the clamped in-plane offsets and the in-box flags once.
    int xoff[XR], qoff[QR];
    unsigned okxy = 0;
#pragma unroll
    for (int q = 0; q < XR; q++) {
        const int e = min(tid + q * NT, PN - 1);
        const int gx = gx0 + e % PX, gy = gy0 + e / PX;
        const bool in = (tid + q * NT < PN) && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        okxy |= (unsigned)in << q;
        xoff[q] = min(max(gy, 0), ny - 1) * nx + min(max(gx, 0), nx - 1);
    }
#pragma unroll
    for (int q = 0; q < QR; q++) {
        const int e = min(tid + q * NT, QN - 1);
        const int gx = gx0 + 1 + e % QX, gy = gy0 + 1 + e / QX;
        const bool in = (tid + q * NT < QN) && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        okxy |= (unsigned)in << (XR + q);
        qoff[q] = min(max(gy, 0), ny - 1) * nx + min(max(gx, 0), nx - 1);
    }

    const T *xsrc = xin ? xin : f;  // any valid array of the same shape when x starts at zero
    // global -> registers for plane k.  Loads are unconditional (clamped
    // addresses); validity is applied at commit, so issuing never waits.
    auto fetch = [&](PlaneRegs<T, FINE> &r, int k) {
        const bool kin = k >= 0 && k < nz && k <= z1 + 1;
        const size_t base = (size_t)min(max(k, 0), nz - 1) * plane;
        r.ok = kin ? okxy : 0u;
        if (!xin) r.ok &= ~((1u << XR) - 1u);  // zero iterate: loaded values are discarded
#pragma unroll
        for (int q = 0; q < XR; q++) r.x[q] = xsrc[base + xoff[q]];
#pragma unroll
        for (int q = 0; q < QR; q++) {
            if constexpr (FINE) r.d[q] = code[base + qoff[q]];
            else r.d[q] = dco[base + qoff[q]];
            r.f[q] = f[base + qoff[q]];
        }
    };
    // registers -> LDS ring slot of plane k (zeros where invalid)
    auto slot3 = [](int k) { return (k + 3) % 3; };  // k >= -2
    auto commit = [&](const PlaneRegs<T, FINE> &r, int k) {
        T *dx = sx[k & 3];
        T *df = sf[slot3(k)];
        DT *dd = sd[slot3(k)];
#pragma unroll
        for (int q = 0; q < XR; q++) {
            const int e = tid + q * NT;
            if (e < PN) dx[e] = ((r.ok >> q) & 1u) ? r.x[q] : T(0);
        }
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const int e = tid + q * NT;
            if (e < QN) {
                const bool ok = (r.ok >> (XR + q)) & 1u;
                df[e] = ok ? r.f[q] : T(0);
                if constexpr (FINE) dd[e] = ok ? r.d[q] : CODE_OFF;
                else dd[e] = ok ? r.d[q] : T(0);
            }
        }
    };

    // Relax colour `col` of plane k on [lo, PX-lo) x [lo, PY-lo) (x-plane coords).
    auto relax = [&](int k, int col, int lo) {
        if (k < 0 || k >= nz) return;
        T *c = sx[k & 3];
        const T *dn = sx[(k - 1) & 3];
        const T *up = sx[(k + 1) & 3];
        const T *fq = sf[slot3(k)];
        const DT *dq = sd[slot3(k)];
        const int half = (PX - 2 * lo) >> 1;
        const int rows = PY - 2 * lo;
        for (int e = tid; e < half * rows; e += NT) {
            const int v = lo + e / half;
            const int u = lo + ((col + gy0 + v + k + gx0 + lo) & 1) + 2 * (e % half);
            const int qq = (v - 1) * QX + (u - 1);
            T d;
            if constexpr (FINE) {
                const uint8_t cd = dq[qq];
                if (cd == CODE_OFF) continue;  // inactive or outside the box
                d = T(12 - (int)cd);
            } else {
                d = dq[qq];
                if (d == T(0)) continue;  // inactive or outside the box
            }
            const int q = v * PX + u;
            const T s = (c[q - 1] + c[q + 1]) + (c[q - PX] + c[q + PX]) + (dn[q] + up[q]);
            c[q] = (s - h2 * fq[qq]) / d;
        }
    };

    auto store = [&](int k) {
        const T *c = sx[k & 3];
        for (int e = tid; e < BX * BY; e += NT) {
            const int u = 2 + e % BX, v = 2 + e / BX;
            const int gx = gx0 + u, gy = gy0 + v;
            if (gx < nx && gy < ny) xout[(size_t)k * plane + (size_t)gy * nx + gx] = c[v * PX + u];
        }
    };

    // Fully unrolled march over at most SEGZ planes (shorter items skip the
    // stores past z1): planes z0-2 .. z0+SEGZ+1 are committed one per step,
    // each refilled register set fetching the plane PF steps ahead, so PF
    // planes of loads stay in flight and every wait count is exact.
    constexpr int NSTEP = SEGZ + 4;
    PlaneRegs<T, FINE> r[PF];
#pragma unroll
    for (int q = 0; q < PF; q++) fetch(r[q], z0 - 2 + q);
#pragma unroll
    for (int st = 0; st < NSTEP; st++) {
        const int pk = z0 - 2 + st;  // plane committed in this step
        commit(r[st % PF], pk);
        if (st + PF < NSTEP) fetch(r[st % PF], pk + PF);
        __syncthreads();
        if (st == 3) {
            relax(z0 - 1, 0, 1);
            relax(z0, 0, 1);
            __syncthreads();
        } else if (st > 3) {
            const int k = pk - 2;
            relax(k + 1, 0, 1);
            __syncthreads();
            relax(k, 1, 2);
            __syncthreads();
            if (k < z1) store(k);
        }
    }
}

}  // namespace rb
}  // namespace mg
