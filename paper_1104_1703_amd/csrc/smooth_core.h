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

// LDS of one work item: a 5-plane ring of x (2-cell halo), and 4-plane rings
// of f and the diagonal (1-cell halo; the finest level keeps its 1-byte
// neighbour code instead of a diagonal).  One ring plane more than a step
// touches lets a step commit its new plane while the previous step's black
// half-sweep may still read the oldest one, so a step needs two barriers.
constexpr int XS = 5, FS = 4;
template <typename T, bool FINE>
struct RbgsLds {
    using DT = typename std::conditional<FINE, uint8_t, T>::type;
    T x[XS][PN];
    T f[FS][QN];
    DT d[FS][QN];
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
    auto xslot = [](int k) { return (k + 2 * XS) % XS; };  // k >= -2
    auto fslot = [](int k) { return (k + 2 * FS) % FS; };
    auto commit = [&](const PlaneRegs<T, FINE> &r, int k) {
        T *dx = sx[xslot(k)];
        T *df = sf[fslot(k)];
        DT *dd = sd[fslot(k)];
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
        T *c = sx[xslot(k)];
        const T *dn = sx[xslot(k - 1)];
        const T *up = sx[xslot(k + 1)];
        const T *fq = sf[fslot(k)];
        const DT *dq = sd[fslot(k)];
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
        const T *c = sx[xslot(k)];
        for (int e = tid; e < BX * BY; e += NT) {
            const int u = 2 + e % BX, v = 2 + e / BX;
            const int gx = gx0 + u, gy = gy0 + v;
            if (gx < nx && gy < ny) xout[(size_t)k * plane + (size_t)gy * nx + gx] = c[v * PX + u];
        }
    };

    // Fully unrolled march over at most SEGZ planes (shorter items skip the
    // stores past z1): planes z0-2 .. z0+SEGZ+1 are committed one per step,
    // each refilled register set fetching the plane PF steps ahead, so PF
    // planes of loads stay in flight and every wait count is exact.  Step k+2
    // commits plane k+2, relaxes red of plane k+1 and stores plane k-1 (black
    // since the previous step), then relaxes black of plane k; the last step
    // only stores.
    constexpr int NSTEP = SEGZ + 4;
    PlaneRegs<T, FINE> r[PF];
#pragma unroll
    for (int q = 0; q < PF; q++) fetch(r[q], z0 - 2 + q);
#pragma unroll
    for (int st = 0; st <= NSTEP; st++) {
        const int pk = z0 - 2 + st;  // plane committed in this step
        const int k = pk - 2;
        if (st < NSTEP) {
            commit(r[st % PF], pk);
            if (st + PF < NSTEP) fetch(r[st % PF], pk + PF);
        }
        __syncthreads();
        if (st == 3) {
            relax(z0 - 1, 0, 1);
            relax(z0, 0, 1);
        } else if (st > 3) {
            if (st < NSTEP) relax(k + 1, 0, 1);
            if (k - 1 >= z0 && k - 1 < z1) store(k - 1);
        }
        if (st > 3 && st < NSTEP) {
            __syncthreads();
            relax(k, 1, 2);
        }
    }
}

}  // namespace rb
}  // namespace mg
