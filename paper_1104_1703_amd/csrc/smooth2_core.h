// Two red-black passes in one march over a work item: temporal blocking of
// the smoother's sweeps (Sec. 2 relaxation, Sec. 3 operator).
//
// A single pass (smooth_core.h) reads x, f and the diagonal of every active
// cell once and writes x once.  Two passes done in one march read and write
// them once for both passes.  The item keeps a 4-cell halo in x and y and
// relaxes four half-sweeps one plane apart as it marches up z: at step st it
// commits plane st (positions count from z0 - 4), then relaxes the first
// pass's red cells on plane st-1 (tile + 3-cell ring), the first pass's black
// cells on plane st-2 (tile + 2), the second pass's red cells on plane st-3
// (tile + 1) and the second pass's black cells on plane st-4 (the tile),
// with a barrier between the four, and stores plane st-5.  Each ring is one
// cell narrower than the one before because a relaxation reads the other
// colour one cell further out; the z planes shift the same way.  Every cell
// of the tile is relaxed from exactly the values two separate passes give
// it, in the same arithmetic, so the result equals two single passes bit for
// bit; the halo cells are recomputed redundantly by neighbouring items.
#pragma once

#include "smooth_core.h"

namespace mg {
namespace rb2 {

using rb::NT;
constexpr int H = 4;  // x halo of two passes
constexpr int BX = TX, BY = TY;
constexpr int PX = BX + 2 * H, PY = BY + 2 * H, PN = PX * PY;  // x plane (40 x 16)
constexpr int QX = PX - 2, QY = PY - 2, QN = QX * QY;          // f / diagonal plane from (1, 1) (38 x 14)
constexpr int XR = (PN + NT - 1) / NT;                         // x elements per thread per plane
constexpr int QR = (QN + NT - 1) / NT;                         // f elements per thread per plane
// Ring depths: a step touches x planes st-5 .. st and f planes st-4 .. st-1;
// the next step's commit may run while slower threads still finish the last
// half-sweep (no barrier at the end of a step), hence one slot more each.
constexpr int XS = 7, FS = 5, CS = 4;
constexpr int CX = BX / 2 + 6, CY = BY / 2 + 6, CPN = CX * CY;  // coarse footprint (PRO), 22 x 10
static_assert(CPN <= NT, "one coarse element per thread");
constexpr int MAXPL = SEG_TILES_FINE * TZ + 2 * H;  // planes of the longest work item with its halo
constexpr int PF64 = 3, PF32 = 4, PFC = 3;

// Activity masks of a fused work item: one word per plane z0-4 .. z0+SEGZ+3,
// bit 4 v + g set when row y0-4+v (0 <= v < 16) holds an active cell in
// granule g of the row (granules as the single-pass masks: x0-16..x0-1,
// x0..x0+15, x0+16..x0+31, x0+32..x0+47).  (u, v): cell (x0-4+u, y0-4+v).
__host__ __device__ constexpr int mask_bit(int u, int v) { return 4 * v + ((u + 16 - H) >> 4); }
static_assert(mask_bit(PX - 1, PY - 1) < 64, "one 64-bit word per plane");

template <typename T, bool FINE, bool PRO>
struct Lds {
    using DT = typename std::conditional<FINE, uint8_t, T>::type;
    static constexpr int DS = PRO ? XS : FS, DN = PRO ? PN : QN;  // PRO: the diagonal rides with x
    T x[XS][PN];
    T f[FS][QN];
    DT d[DS][DN];
    unsigned long long m[MAXPL];
    T c[PRO ? CS : 1][PRO ? CPN : 1];
};

template <typename T, bool FINE, bool PRO>
struct Regs {
    using DT = typename std::conditional<FINE, uint8_t, T>::type;
    T x[XR];
    T f[QR];
    DT d[PRO ? XR : QR];
};

// Two red-black passes over one work item: xin -> xout (xin == nullptr reads
// zero).  Called by all NT threads of a block.  pm: the item's SEGZ + 8 masks
// (mask_bit layout).  PRO: the first pass starts from x + P2(xc) on active
// cells, as the single prolongation pass does (xc: level + 1, cnx x cny x cnz;
// x0, y0, z0 even).
template <typename T, bool FINE, int SEGZ, bool PRO = false>
__device__ __forceinline__ void rbgs2_item(Lds<T, FINE, PRO> &L, const T *__restrict__ xin, T *__restrict__ xout,
                                           const T *__restrict__ f, const uint8_t *__restrict__ code,
                                           const T *__restrict__ dco, int nx, int ny, int nz, T h2, const Seg sg,
                                           const unsigned long long *__restrict__ pm,
                                           const T *__restrict__ xc = nullptr, int cnx = 0, int cny = 0,
                                           int cnz = 0) {
    static_assert(SEGZ + 2 * H <= MAXPL, "work item longer than the mask array");
    static_assert(FINE || !PRO, "coarse levels prolong with the single-pass kernel");
    using DT = typename Lds<T, FINE, PRO>::DT;
    using R = Regs<T, FINE, PRO>;
    constexpr int DS = Lds<T, FINE, PRO>::DS;
    auto &sx = L.x;
    auto &sf = L.f;
    auto &sd = L.d;
    const int gx0 = sg.x0 - H, gy0 = sg.y0 - H;  // origin of the x plane
    const size_t plane = (size_t)nx * ny;
    const int tid = threadIdx.x;
    const int z0 = max(sg.z0, 0), z1 = min(sg.z1, nz);
    constexpr int NP = SEGZ + 2 * H;  // planes z0-4 .. z0+SEGZ+3

    if (tid < NP) L.m[tid] = pm[tid];

    int xoff[XR], qoff[QR];
    unsigned long long bits = 0;  // 8 bits per element: its mask bit
#pragma unroll
    for (int q = 0; q < XR; q++) {
        const int e = min(tid + q * NT, PN - 1);
        const int u = e % PX, v = e / PX;
        const int gx = gx0 + u, gy = gy0 + v;
        const bool in = (tid + q * NT < PN) && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        xoff[q] = in ? (gy * nx + gx) * (int)sizeof(T) : OFF_NONE;
        bits |= (unsigned long long)mask_bit(u, v) << (8 * q);
    }
#pragma unroll
    for (int q = 0; q < QR; q++) {
        const int e = min(tid + q * NT, QN - 1);
        const int u = e % QX + 1, v = e / QX + 1;
        const int gx = gx0 + u, gy = gy0 + v;
        const bool in = (tid + q * NT < QN) && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
        qoff[q] = in ? (gy * nx + gx) * (int)sizeof(T) : OFF_NONE;
        bits |= (unsigned long long)mask_bit(u, v) << (8 * (XR + q));
    }
    static_assert(XR + QR <= 8, "mask bit indices are packed into one 64-bit word");
    const int pbytes = (int)(plane * sizeof(T));
    constexpr int TSH = sizeof(T) == 8 ? 3 : 2;

    // PRO: the coarse footprint element of this thread (coarse plane ck =
    // K - (z0/2 - 3) >= 0), as in the single prolongation pass
    const int cI0 = sg.x0 / 2 - 3, cJ0 = sg.y0 / 2 - 3, cK0 = z0 / 2 - 3;
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

    // global -> registers for step st: x of plane position st (plane
    // z0-4+st, planes z0-4 .. z1+3) and f and the diagonal of position st-1
    // (planes z0-3 .. z1+2); PRO loads the diagonal with x
    auto fetch = [&](R &r, int st) {
        const int kx = z0 - H + st;
        const bool xk = kx >= 0 && kx < nz && kx <= z1 + H - 1;
        const unsigned long long mx = xk ? L.m[st] : 0ull;
        const size_t bx = (size_t)min(max(kx, 0), nz - 1) * plane;
        const __amdgpu_buffer_rsrc_t rx = rsrc(xin ? xin + bx : f + bx, xin ? pbytes : 0);
#pragma unroll
        for (int q = 0; q < XR; q++) {
            const int o = mbit(mx, q) ? xoff[q] : OFF_NONE;
            r.x[q] = bload<T>(rx, o);
            if constexpr (PRO) r.d[q] = bload<uint8_t>(rsrc(code + bx, (int)plane), o == OFF_NONE ? o : o >> TSH);
        }
        const int kf = kx - 1;
        const bool fk = st >= 2 && kf >= 0 && kf < nz && kf <= z1 + H - 2;  // positions 1 .. NP-2
        const unsigned long long mf = fk ? L.m[st >= 1 ? st - 1 : 0] : 0ull;
        const size_t bf = (size_t)min(max(kf, 0), nz - 1) * plane;
        const __amdgpu_buffer_rsrc_t rf = rsrc(f + bf, pbytes);
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const bool p = qoff[q] != OFF_NONE && mbit(mf, XR + q);
            r.f[q] = bload<T>(rf, p ? qoff[q] : OFF_NONE);
            if constexpr (!PRO) {
                if constexpr (FINE) r.d[q] = bload<uint8_t>(rsrc(code + bf, (int)plane), p ? qoff[q] >> TSH : OFF_NONE);
                else r.d[q] = bload<T>(rsrc(dco + bf, pbytes), p ? qoff[q] : OFF_NONE);
            }
        }
    };
    // diagonal of x-plane cell (u, v) in its ring plane
    auto didx = [](int u, int v) { return PRO ? v * PX + u : (v - 1) * QX + (u - 1); };
    auto dslot = [](int P) { return P % DS; };
    // registers -> LDS for step st (skipped loads read zero, which is also
    // the code of an inactive cell)
    auto commit = [&](const R &r, int st) {
        T *dx = sx[st % XS];
#pragma unroll
        for (int q = 0; q < XR; q++) {
            const int e = tid + q * NT;
            if (e >= PN) continue;
            T xv = r.x[q];
            if constexpr (PRO) {
                sd[dslot(st)][e] = r.d[q];
                if (r.d[q] != DT(0)) {
                    // P2: parents (I + a sx, J + b sy, K + c sz), weights 3/4 and
                    // 1/4 per axis, summed in the order of the prolongation kernels
                    const int u = e % PX, v = e / PX;
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
        if (st >= 1) {
            T *df = sf[(st - 1) % FS];
#pragma unroll
            for (int q = 0; q < QR; q++) {
                const int e = tid + q * NT;
                if (e < QN) {
                    df[e] = r.f[q];
                    if constexpr (!PRO) sd[dslot(st - 1)][e] = r.d[q];
                }
            }
        }
    };
    // Relax colour col of plane position P (plane z0-4+P) on
    // [lo, PX-lo) x [lo, PY-lo) in x-plane coordinates, as the single pass does.
    auto relax = [&](int P, int col, int lo) {
        const int k = z0 - H + P;
        if (k < 0 || k >= nz) return;
        T *c = sx[P % XS];
        const T *dn = sx[(P - 1) % XS];
        const T *up = sx[(P + 1) % XS];
        const T *fq = sf[P % FS];
        const DT *dq = sd[dslot(P)];
        const int half = (PX - 2 * lo) >> 1;
        const int rows = PY - 2 * lo;
        for (int e = tid; e < half * rows; e += NT) {
            const int v = lo + e / half;
            const int u = lo + ((col + gy0 + v + k + gx0 + lo) & 1) + 2 * (e % half);
            const int qq = (v - 1) * QX + (u - 1);
            T d;
            if constexpr (FINE) d = T((int)dq[didx(u, v)]);
            else d = dq[didx(u, v)];
            if (d == T(0)) continue;
            const int q = v * PX + u;
            const T s = (c[q - 1] + c[q + 1]) + (c[q - PX] + c[q + PX]) + (dn[q] + up[q]);
            c[q] = (s - h2 * fq[qq]) / d;
        }
    };
    // LDS -> xout for the tile cells of plane position P; inactive cells are
    // not written (they hold zero in every iterate buffer)
    auto store = [&](int P) {
        const int k = z0 - H + P;
        const T *c = sx[P % XS];
        const DT *dq = sd[dslot(P)];
        const __amdgpu_buffer_rsrc_t ro = rsrc(xout + (size_t)k * plane, pbytes);
        for (int e = tid; e < BX * BY; e += NT) {
            const int u = H + e % BX, v = H + e / BX;
            const int gx = gx0 + u, gy = gy0 + v;
            const bool act = dq[didx(u, v)] != DT(0);
            bstore<T>(c[v * PX + u], ro, act ? (gy * nx + gx) * (int)sizeof(T) : OFF_NONE);
        }
    };

    constexpr int PF = !FINE ? (PFC < NP ? PFC : NP) : sizeof(T) == 8 ? PF64 : PF32;
    constexpr int CKMAX = ((NP - 1) >> 1) + 2;  // last coarse plane read (PRO)
    R r[PF];
#pragma unroll
    for (int q = 0; q < PF; q++) fetch(r[q], q);
#pragma unroll
    for (int st = 0; st <= NP; st++) {
        if (st < NP) {
            if constexpr (PRO) {
                // an odd step stores coarse plane st/2 + 3 for the next commits
                // (its ring slot was last read two steps before)
                if ((st & 1) && (st >> 1) + 3 <= CKMAX) {
                    const int P = (st >> 1) + 3;
                    if (tid < CPN) L.c[P % CS][tid] = cr[(st >> 1) & 1];
                    if (P + 2 <= CKMAX) cr[(st >> 1) & 1] = cload(P + 2);
                }
            }
            commit(r[st % PF], st);
            if (st + PF < NP) fetch(r[st % PF], st + PF);
        }
        __syncthreads();
        if (st - 1 >= 1 && st - 1 <= NP - 2) relax(st - 1, 0, 1);  // first pass, red
        if (st - 5 >= H && st - 5 <= NP - 1 - H && z0 - H + (st - 5) < z1) store(st - 5);
        if (st - 2 >= 2 && st - 2 <= NP - 3) {
            __syncthreads();
            relax(st - 2, 1, 2);  // first pass, black
        }
        if (st - 3 >= 3 && st - 3 <= NP - 4) {
            __syncthreads();
            relax(st - 3, 0, 3);  // second pass, red
        }
        if (st - 4 >= 4 && st - 4 <= NP - 5) {
            __syncthreads();
            relax(st - 4, 1, 4);  // second pass, black
        }
    }
}

}  // namespace rb2
}  // namespace mg
