// Core of the red-black smoother, shared by the per-level kernels
// (smooth.hip) and the batched phase kernels (batch.hip).
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include "masked.h"
#include "tiles.h"

namespace mg {
namespace rb {


constexpr int BX = TX, BY = TY;
constexpr int PX = BX + 4, PY = BY + 4, PN = PX * PY;  // x plane with 2-cell halo
constexpr int QX = BX + 2, QY = BY + 2, QN = QX * QY;  // f / diag plane with 1-cell halo
constexpr int NT = 256;
constexpr int XR = (PN + NT - 1) / NT;  // x elements per thread per plane
constexpr int QR = (QN + NT - 1) / NT;  // f elements per thread per plane
// Planes of global loads in flight per block.  Double planes carry twice the
// bytes of float planes; measured on the 256^3 workload, three are best for
// doubles and more would only keep lines in L2 longer; three for floats (two
// in the pass that applies the prolongation) let the finest float passes run
// eight blocks per CU without spills (four at five blocks: plain pass 34.6
// against 30.1 us, prolongation pass 46.0 against 41.3 us at three).
constexpr int PF64 = 3, PF32 = 3;
constexpr int PFC = 3;  // coarse levels

// Work items are dealt to the 8 XCDs round-robin by block id; give each XCD a
// contiguous range of work items so that halo re-reads hit its own L2.
__device__ __forceinline__ int xcd_item(int b, int nb) {
    const int per = nb >> 3;  // nb is a multiple of 8
    return (b & 7) * per + (b >> 3);
}

// PRO: the pass starts with the P2 prolongation and correction x += P2(xc)
// applied to every plane as it enters LDS (the first post-smoothing pass); the
// diagonal or code is then kept on the whole x plane (the 2-cell halo must be
// known inactive to stay zero).
template <typename T, bool FINE, bool PRO>
struct PlaneRegs {
    T x[XR];
    T f[QR];
    typename std::conditional<FINE, uint8_t, T>::type d[PRO ? XR : QR];  // raw code byte or diagonal
};

// LDS of one work item: a 5-plane ring of x (2-cell halo), and 4-plane rings
// of f and the diagonal (1-cell halo; the finest level keeps its 1-byte
// neighbour code instead of a diagonal).  One ring plane more than a step
// touches lets a step commit its new plane while the previous step's black
// half-sweep may still read the oldest one, so a step needs two barriers.
// `m` holds the item's activity masks, one word per plane (see item_mask_bit).
// With PRO, `c` is a 4-plane ring of the coarse footprint of the x plane
// (CX x CY coarse cells at (x0/2 - 2, y0/2 - 2)).
constexpr int CS = 4;
// Ring depths.  Coarse FP64 levels use one plane less in each ring and a
// third barrier per step (after the black half-sweep), which keeps a block
// under 32 KB of LDS: five blocks per CU, so a level-1 pass fits in one round.
template <typename T, bool FINE>
struct Rings {
    static constexpr bool SLIM = !FINE && sizeof(T) == 8;
    static constexpr int XS = SLIM ? 4 : 5, FS = SLIM ? 3 : 4;
};
constexpr int CX = BX / 2 + 4, CY = BY / 2 + 4, CPN = CX * CY;
static_assert(CPN <= NT, "one coarse element per thread");
constexpr int MAXPL = SEGZ_FINE_MAX + 4;  // planes touched by the longest work item
template <typename T, bool FINE, bool PRO = false>
struct RbgsLds {
    using DT = typename std::conditional<FINE, uint8_t, T>::type;
    static constexpr int DN = PRO ? PN : QN;
    static constexpr int XS = Rings<T, FINE>::XS, FS = Rings<T, FINE>::FS;
    T x[XS][PN];
    T f[FS][QN];
    DT d[FS][DN];
    unsigned long long m[MAXPL];
    T c[PRO ? CS : 1][PRO ? CPN : 1];
    T rcp[FINE ? 16 : 1];  // finest level: correctly rounded 1/d for the diagonals d = 1..12
};

// Correctly rounded reciprocals of 1..12 (constant-folded at compile time
// with IEEE division in each precision).
constexpr double RCP64[13] = {0.0,       1.0,       1.0 / 2,  1.0 / 3,  1.0 / 4,  1.0 / 5, 1.0 / 6,
                              1.0 / 7,   1.0 / 8,   1.0 / 9,  1.0 / 10, 1.0 / 11, 1.0 / 12};
constexpr float RCP32[13] = {0.0f,      1.0f,      1.0f / 2, 1.0f / 3, 1.0f / 4,  1.0f / 5,  1.0f / 6,
                             1.0f / 7,  1.0f / 8,  1.0f / 9, 1.0f / 10, 1.0f / 11, 1.0f / 12};

// a / d with y = RN(1/d) (the finest level's diagonals 1..12 from a table,
// coarse diagonals from one division per cell and call): q0 = RN(a y) is
// within one unit in the last place of a/d, the remainder a - q0 d is exact
// under a fused multiply-add, and one correction step q0 + (a - q0 d) y
// rounds to the correctly rounded quotient (Markstein's theorem), so the
// result is bit for bit that of the division, except that a quotient in the
// subnormal range may differ from it by one unit of that range.  The
// remainder is formed as -(q0 d - a) so that a zero keeps its sign.
template <typename T>
__device__ __forceinline__ T div_small(T a, T d, T y) {
    const T q0 = a * y;
    const T r = -__builtin_fma(q0, d, -a);
    return __builtin_fma(r, y, q0);
}

// One full red-black pass over one work item (see the file comment of
// smooth.hip).  Called by all 256 threads of a block.  `pm`: the item's
// SEGZ + 4 activity masks, or nullptr to load every in-box cell.  A plane of
// the level must hold fewer than 2^31 bytes.  PRO: xc is the next coarser
// level's iterate (cnx x cny x cnz); the item's x0, y0 and z0 are even.
// NORMIN (finest level): the pass also returns the thread's sum over the
// item's planes of r^2, r = (L xin - f) at its own tile cell, the residual
// of the pass's input.  A plane committed at step st is not relaxed before
// step st + 1, so right after the step's first barrier each thread reads its
// cell and the four in-plane neighbours there; with the two planes before
// it in registers, the residual of the plane below is formed with the same
// expression and plane order as the residual-norm march, so the block sums
// are bit for bit the march's.
template <typename T, bool FINE, int SEGZ, bool PRO = false, bool NORMIN = false>
__device__ __forceinline__ double rbgs_item(RbgsLds<T, FINE, PRO> &L, const T *__restrict__ xin,
                                            T *__restrict__ xout, const T *__restrict__ f,
                                            const uint8_t *__restrict__ code, const T *__restrict__ dco, int nx,
                                            int ny, int nz, T h2, const Seg sg,
                                            const unsigned long long *__restrict__ pm,
                                            const T *__restrict__ xc = nullptr, int cnx = 0, int cny = 0,
                                            int cnz = 0, T ih2 = T(0)) {
    static_assert(SEGZ + 4 <= MAXPL, "work item longer than the mask array");
    static_assert(!NORMIN || (FINE && !PRO), "the input residual is formed on the finest level only");
    using DT = typename RbgsLds<T, FINE, PRO>::DT;
    using Regs = PlaneRegs<T, FINE, PRO>;
    constexpr bool SLIM = Rings<T, FINE>::SLIM;
    constexpr int XS = Rings<T, FINE>::XS, FS = Rings<T, FINE>::FS;
    auto &sx = L.x;
    auto &sf = L.f;
    auto &sd = L.d;
    const int gx0 = sg.x0 - 2, gy0 = sg.y0 - 2;  // origin of the x plane (2-cell halo)
    const size_t plane = (size_t)nx * ny;
    const int tid = threadIdx.x;
    const int z0 = max(sg.z0, 0), z1 = min(sg.z1, nz);  // a work item never leaves the box

    if (tid < SEGZ + 4) L.m[tid] = pm ? pm[tid] : ~0ull;
    if constexpr (FINE && !NORMIN)
        if (tid < 16) L.rcp[tid] = tid <= 12 ? T(sizeof(T) == 8 ? RCP64[tid] : RCP32[tid]) : T(0);

    // Per-thread element positions are the same for every plane: precompute
    // the in-plane byte offsets (OFF_NONE outside the box) and the mask bits
    // of the thread's elements (one byte each) once.
    int xoff[XR], qoff[QR];
    unsigned bits = 0;
#pragma unroll
    for (int q = 0; q < XR; q++) {
        const int e = min(tid + q * NT, PN - 1);
        const int u = e % PX, v = e / PX;
        const int gx = gx0 + u, gy = gy0 + v;
        const bool in = (tid + q * NT < PN) && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        xoff[q] = in ? (gy * nx + gx) * (int)sizeof(T) : OFF_NONE;
        bits |= (unsigned)item_mask_bit(u, v) << (8 * q);
    }
#pragma unroll
    for (int q = 0; q < QR; q++) {
        const int e = min(tid + q * NT, QN - 1);
        const int u = e % QX + 1, v = e / QX + 1;
        const int gx = gx0 + u, gy = gy0 + v;
        const bool in = (tid + q * NT < QN) && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        qoff[q] = in ? (gy * nx + gx) * (int)sizeof(T) : OFF_NONE;
        bits |= (unsigned)item_mask_bit(u, v) << (8 * (XR + q));
    }
    static_assert(XR + QR <= 4, "mask bit indices are packed into one word");
    const int pbytes = (int)(plane * sizeof(T));
    constexpr int TSH = sizeof(T) == 8 ? 3 : 2;  // byte offset -> element offset

    // PRO: coarse footprint element of this thread and the coarse plane loads
    // (coarse plane index ck = K - (z0/2 - 2) >= 0)
    const int cI0 = sg.x0 / 2 - 2, cJ0 = sg.y0 / 2 - 2, cK0 = z0 / 2 - 2;
    int coff = OFF_NONE;
    if constexpr (PRO) {
        const int ci = cI0 + tid % CX, cj = cJ0 + tid / CX;
        if (tid < CPN && ci >= 0 && ci < cnx && cj >= 0 && cj < cny) coff = (cj * cnx + ci) * (int)sizeof(T);
    }
    const size_t cpl = (size_t)cnx * cny;
    auto cload = [&](int ck) -> T {
        const int K = cK0 + ck;
        if (!PRO || K < 0 || K >= cnz) return T(0);
        return bload<T>(rsrc(xc + (size_t)K * cpl, (int)(cpl * sizeof(T))), coff);
    };
    T cr[2] = {T(0), T(0)};
    if constexpr (PRO) {
        const T c0 = cload(0), c1 = cload(1), c2 = cload(2);
        if (tid < CPN) {
            L.c[0][tid] = c0;
            L.c[1][tid] = c1;
            L.c[2][tid] = c2;
        }
        cr[0] = cload(3);
        cr[1] = cload(4);
    }
    __syncthreads();  // masks (and the first coarse planes)

    auto mbit = [&](unsigned long long m, int j) { return (bool)((m >> ((bits >> (8 * j)) & 63u)) & 1ull); };
    // f and the diagonal are read on planes z0-1 .. z1 only
    auto fplane = [&](int k) { return k >= z0 - 1 && k <= z1 && k < nz; };
    auto fload = [&](unsigned long long m, int k, int q) { return fplane(k) && qoff[q] >= 0 && mbit(m, XR + q); };

    // global -> registers for plane k = z0 - 2 + pi (x on planes z0-2 .. z1+1)
    auto fetch = [&](Regs &r, int k, int pi) {
        const bool kin = k >= 0 && k < nz && k <= z1 + 1;
        const unsigned long long m = kin ? L.m[pi] : 0ull;
        const size_t base = (size_t)min(max(k, 0), nz - 1) * plane;
        const __amdgpu_buffer_rsrc_t rx = rsrc(xin ? xin + base : f + base, xin ? pbytes : 0);
        const __amdgpu_buffer_rsrc_t rf = rsrc(f + base, pbytes);
#pragma unroll
        for (int q = 0; q < XR; q++) {
            const int o = mbit(m, q) ? xoff[q] : OFF_NONE;
            r.x[q] = bload<T>(rx, o);
            if constexpr (PRO) {  // the diagonal on the whole x plane
                if constexpr (FINE) r.d[q] = bload<uint8_t>(rsrc(code + base, (int)plane), o == OFF_NONE ? o : o >> TSH);
                else r.d[q] = bload<T>(rsrc(dco + base, pbytes), o);
            }
        }
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const bool p = fload(m, k, q);
            r.f[q] = bload<T>(rf, p ? qoff[q] : OFF_NONE);
            if constexpr (!PRO) {
                if constexpr (FINE) r.d[q] = bload<uint8_t>(rsrc(code + base, (int)plane), p ? qoff[q] >> TSH : OFF_NONE);
                else r.d[q] = bload<T>(rsrc(dco + base, pbytes), p ? qoff[q] : OFF_NONE);
            }
        }
    };
    // Ring slots are indexed by a plane's position j = k - z0 in the item
    // (j >= -2), a compile-time value in the unrolled march.
    auto xslot = [](int j) { return (j + 2 * XS) % XS; };
    auto fslot = [](int j) { return (j + 2 * FS) % FS; };
    // diagonal of x-plane cell (u, v) in its ring plane
    auto didx = [](int u, int v) { return PRO ? v * PX + u : (v - 1) * QX + (u - 1); };
    // registers -> LDS ring slot of plane z0 + j (skipped loads read zero,
    // which is also the code of an inactive cell); st = j + 2 is the step
    auto commit = [&](const Regs &r, int j) {
        T *dx = sx[xslot(j)];
        T *df = sf[fslot(j)];
        DT *dd = sd[fslot(j)];
#pragma unroll
        for (int q = 0; q < XR; q++) {
            const int e = tid + q * NT;
            if (e >= PN) continue;
            T xv = r.x[q];
            if constexpr (PRO) {
                dd[e] = r.d[q];
                if (r.d[q] != DT(0)) {
                    // P2: parents (I + a sx, J + b sy, K + c sz) with weights 3/4, 1/4
                    // per axis, summed in the order of the prolongation kernels
                    const int u = e % PX, v = e / PX, st = j + 2;
                    const int a0 = 1 + (u >> 1), b0 = 1 + (v >> 1);
                    const int sxx = (u & 1) ? 1 : -1, syy = (v & 1) ? 1 : -1;
                    const int ck0 = 1 + (st >> 1), ck1 = ck0 + ((st & 1) ? 1 : -1);
                    const T w4[2] = {T(0.75), T(0.25)};
                    T s = T(0);
#pragma unroll
                    for (int cz = 0; cz < 2; cz++) {
                        const T *cp = L.c[(cz ? ck1 : ck0) % CS];
#pragma unroll
                        for (int b = 0; b < 2; b++)
#pragma unroll
                            for (int a = 0; a < 2; a++)
                                s += w4[a] * w4[b] * w4[cz] * cp[(b0 + b * syy) * CX + (a0 + a * sxx)];
                    }
                    xv = xv + s;
                }
            }
            dx[e] = xv;
        }
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const int e = tid + q * NT;
            if (e < QN) {
                df[e] = r.f[q];
                if constexpr (!PRO) dd[e] = r.d[q];
            }
        }
    };

    // Relax colour `col` of plane k = z0 + j on [lo, PX-lo) x [lo, PY-lo)
    // (x-plane coords).  The diagonal is 0 on inactive and out-of-box cells.
    auto relax = [&](int j, int col, int lo) {
        const int k = z0 + j;
        if (k < 0 || k >= nz) return;
        T *c = sx[xslot(j)];
        const T *dn = sx[xslot(j - 1)];
        const T *up = sx[xslot(j + 1)];
        const T *fq = sf[fslot(j)];
        const DT *dq = sd[fslot(j)];
        const int half = (PX - 2 * lo) >> 1;
        const int rows = PY - 2 * lo;
        for (int e = tid; e < half * rows; e += NT) {
            const int v = lo + e / half;
            const int u = lo + ((col + gy0 + v + k + gx0 + lo) & 1) + 2 * (e % half);
            const int qq = (v - 1) * QX + (u - 1);
            if constexpr (FINE && !NORMIN) {  // (the norm-forming pass has no registers to spare)
                const int ci = (int)dq[didx(u, v)];
                if (ci == 0) continue;
                const int q = v * PX + u;
                const T s = (c[q - 1] + c[q + 1]) + (c[q - PX] + c[q + PX]) + (dn[q] + up[q]);
                c[q] = div_small<T>(s - h2 * fq[qq], T(ci), L.rcp[ci]);
            } else {
                T d;
                if constexpr (FINE) d = T((int)dq[didx(u, v)]);
                else d = dq[didx(u, v)];
                if (d == T(0)) continue;
                const int q = v * PX + u;
                const T s = (c[q - 1] + c[q + 1]) + (c[q - PX] + c[q + PX]) + (dn[q] + up[q]);
                c[q] = (s - h2 * fq[qq]) / d;
            }
        }
    };

    // LDS -> xout for the tile cells of plane z0 + j; inactive cells are not
    // written (they hold zero in every iterate buffer).  The slim rings no
    // longer hold the plane's diagonal here: every in-box cell is written
    // (inactive ones with their zero).
    auto store = [&](int j) {
        const T *c = sx[xslot(j)];
        const DT *dq = sd[fslot(j)];
        const __amdgpu_buffer_rsrc_t ro = rsrc(xout + (size_t)(z0 + j) * plane, pbytes);
        for (int e = tid; e < BX * BY; e += NT) {
            const int u = 2 + e % BX, v = 2 + e / BX;
            const int gx = gx0 + u, gy = gy0 + v;
            bool act;
            if constexpr (SLIM) act = gx < nx && gy < ny;
            else act = dq[didx(u, v)] != DT(0);
            bstore<T>(c[v * PX + u], ro, act ? (gy * nx + gx) * (int)sizeof(T) : OFF_NONE);
        }
    };

    // Fully unrolled march over at most SEGZ planes (shorter items skip the
    // stores past z1): planes z0-2 .. z0+SEGZ+1 are committed one per step,
    // each refilled register set fetching the plane PF steps ahead, so PF
    // planes of loads stay in flight and every wait count is exact.  Step k+2
    // commits plane k+2, relaxes red of plane k+1 and stores plane k-1 (black
    // since the previous step), then relaxes black of plane k; the last step
    // only stores.  PRO: the commit of step st reads coarse planes
    // ck = st/2 .. st/2 + 2; an odd step stores coarse plane st/2 + 3 for the
    // next steps (its ring slot was last read two steps before).
    constexpr int NSTEP = SEGZ + 4;
    constexpr int PF = !FINE ? (PFC < NSTEP ? PFC : NSTEP) : sizeof(T) == 8 ? PF64 : PRO ? PF32 - 1 : PF32;
    constexpr int CKMAX = ((NSTEP - 1) >> 1) + 2;  // last coarse plane read
    Regs r[PF];
#pragma unroll
    for (int q = 0; q < PF; q++) fetch(r[q], z0 - 2 + q, q);
    // NORMIN: own tile cell, its x at the last two positions read, the
    // in-plane neighbour sum of the newer one, and the thread's sum of r^2
    const int q0 = (tid / BX + 2) * PX + (tid % BX + 2);
    const int qf = (tid / BX + 1) * QX + (tid % BX + 1);
    T xa = T(0), xb = T(0), nb = T(0);
    double sq = 0.0;
#pragma unroll
    for (int st = 0; st <= NSTEP; st++) {
        const int j = st - 4;  // plane z0 + j is black-relaxed in this step
        if (st < NSTEP) {
            if constexpr (PRO) {
                if ((st & 1) && (st >> 1) + 3 <= CKMAX) {
                    const int P = (st >> 1) + 3;
                    if (tid < CPN) L.c[P % CS][tid] = cr[(st >> 1) & 1];
                    if (P + 2 <= CKMAX) cr[(st >> 1) & 1] = cload(P + 2);
                }
            }
            commit(r[st % PF], j + 2);
            if (st + PF < NSTEP) fetch(r[st % PF], z0 + j + 2 + PF, st + PF);
        }
        __syncthreads();
        if constexpr (NORMIN) {
            if (st >= 1 && st < NSTEP) {  // position st - 2 was committed in this step
                const T *cp = sx[xslot(st - 2)];
                const T xn = cp[q0];
                const T sn = (cp[q0 - 1] + cp[q0 + 1]) + (cp[q0 - PX] + cp[q0 + PX]);
                if (st >= 3 && st - 3 < z1 - z0) {  // residual of position st - 3
                    const T fv = sf[fslot(st - 3)][qf];
                    const T d = T((int)sd[fslot(st - 3)][qf]);
                    T rr = T(0);
                    if (d != T(0)) rr = ((nb + (xa + xn)) - d * xb) * ih2 - fv;
                    sq += (double)rr * (double)rr;
                }
                xa = xb;
                xb = xn;
                nb = sn;
            }
        }
        if (st == 3) {
            relax(-1, 0, 1);
            relax(0, 0, 1);
        } else if (st > 3) {
            if (st < NSTEP) relax(j + 1, 0, 1);
            if (j - 1 >= 0 && z0 + j - 1 < z1) store(j - 1);
        }
        if (st > 3 && st < NSTEP) {
            __syncthreads();
            relax(j, 1, 2);
        }
        // slim rings: the next commit overwrites a plane this step still read
        if constexpr (SLIM)
            if (st >= 3 && st < NSTEP) __syncthreads();
    }
    return sq;
}

}  // namespace rb
}  // namespace mg
