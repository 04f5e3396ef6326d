// Finest-level red-black pass that also forms the residual of its result and
// the R1 restriction of that residual onto level 1 (Sec. 2: the last
// pre-smoothing pass, then r = L x - f and f_c = -R1 r), so that the residual
// march after the pre-smoothing is not needed.
//
// Same z march over the smoother's work items as the plain pass
// (smooth_core.h), with one more cell of xy halo: x is staged with a 3-cell
// halo, f and the neighbour code with a 2-cell halo.  Red cells are relaxed on
// the tile plus a 2-cell ring and black cells on the tile plus a 1-cell ring,
// so that every in-plane neighbour of a tile cell holds its final value of the
// pass.  A plane is final once its black half-sweep is done; in the black
// phase of the next step each thread reads its own tile cell and the four
// in-plane neighbours of that plane, and with the two final planes before it
// in registers forms the residual of the plane below, in the expression and
// neighbour order of the residual march, then sums the 2 x 2 x 2 children by
// lane exchanges and planes in the march's order.  The iterate, the residual and the restricted
// right-hand side are therefore those of the plain pass followed by the march,
// bit for bit.
#pragma once

#include "smooth_core.h"

namespace mg {
namespace rbr {

using rb::NT;
constexpr int BX = TX, BY = TY;
constexpr int H = 3;                                            // x halo
constexpr int PX = BX + 2 * H, PY = BY + 2 * H, PN = PX * PY;   // 38 x 14
constexpr int QX = BX + 2 * H - 2, QY = BY + 2 * H - 2, QN = QX * QY;  // f / code, 2-cell halo: 36 x 12
constexpr int XR = (PN + NT - 1) / NT;
constexpr int QR = (QN + NT - 1) / NT;
constexpr int MAXPL = SEGZ_FINE_MAX + 2 * H;  // mask words of the longest work item
constexpr int CXN = BX / 2 * (BY / 2);  // coarse cells above one tile plane pair
// Planes of global loads in flight (doubles: two were measured as fast as
// three and take 14 fewer registers; floats: two keep six blocks per CU free
// of spills, 52.3 against 54.7 us with three at five blocks)
constexpr int PF64 = 2, PF32 = 2;
static_assert(BX == 32 && BY * BX == NT, "one tile cell per thread, two tile rows per wave");

// Mask bit of x-plane cell (u, v) (cell (x0-3+u, y0-3+v)) in the item's mask
// words built with a 3-cell halo: bit 4 v + g, g the 16-cell granule of the
// row with boundaries at x0-16, x0, x0+16, x0+32.
__host__ __device__ constexpr int mask_bit(int u, int v) { return 4 * v + ((u + 16 - H) >> 4); }

// LDS of one work item: 5-plane x and 4-plane f / code rings (one plane more
// than a step touches, so a step needs two barriers; 38 KB for doubles, four
// blocks per CU).  Slimmer rings with a third barrier per step fit five
// blocks per CU but were measured slower (with register spills at that
// occupancy).
template <typename T>
struct Lds {
    static constexpr int XS = 5, FS = 4;
    T x[XS][PN];
    T f[FS][QN];
    uint8_t d[FS][QN];
    unsigned long long m[MAXPL];
    T rcp[16];
    uint8_t cf[SEGZ_FINE_MAX / 2][CXN];  // coarse cells above the item: diagonal != 0
};

// One work item, called by all NT threads of a block.  pm: the item's
// SEGZ + 6 mask words (planes z0-3 .. z0+SEGZ+2).  xin may be null (x = 0).
// The item's x0, y0 and z0 are even.  Coarse cells above the item's tile
// columns get f_c = -(1/8) sum of their children's residuals where the coarse
// diagonal cd is non-zero, 0 elsewhere.
template <typename T, int SEGZ>
__device__ __forceinline__ void rbgs_res_item(Lds<T> &L, const T *__restrict__ xin, T *__restrict__ xout,
                                              const T *__restrict__ f, const uint8_t *__restrict__ code, int nx,
                                              int ny, int nz, T h2, T ih2, const Seg sg,
                                              const unsigned long long *__restrict__ pm, const T *__restrict__ cd,
                                              int cnx, int cny, T *__restrict__ fc) {
    static_assert(SEGZ + 2 * H <= MAXPL, "work item longer than the mask array");
    constexpr int XS = Lds<T>::XS, FS = Lds<T>::FS;
    auto &sx = L.x;
    auto &sf = L.f;
    auto &sd = L.d;
    const int gx0 = sg.x0 - H, gy0 = sg.y0 - H;
    const size_t plane = (size_t)nx * ny;
    const int tid = threadIdx.x;
    const int z0 = max(sg.z0, 0), z1 = min(sg.z1, nz);
    const int zlen = z1 - z0;

    if (tid < SEGZ + 2 * H) L.m[tid] = pm[tid];
    if (tid < 16) L.rcp[tid] = tid <= 12 ? T(sizeof(T) == 8 ? rb::RCP64[tid] : rb::RCP32[tid]) : T(0);
    // activity of the coarse cells the item restricts onto, staged once (a
    // load waited for inside the march would also wait for the plane loads
    // in flight before it)
    for (int i = tid; i < SEGZ / 2 * CXN; i += NT) {
        const int c = i % CXN, K = (z0 >> 1) + i / CXN;
        const int cx = (sg.x0 >> 1) + c % (BX / 2), cy = (sg.y0 >> 1) + c / (BX / 2);
        const int cnz = nz >> 1;
        L.cf[i / CXN][c] = cx < cnx && cy < cny && K < cnz && cd[((size_t)K * cny + cy) * cnx + cx] != T(0);
    }

    // per-thread plane elements: in-plane byte offsets (OFF_NONE outside the
    // box) and mask bit indices (one byte each)
    int xoff[XR], qoff[QR];
    unsigned long long bits = 0;
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
    __syncthreads();  // masks

    auto mbit = [&](unsigned long long m, int j) { return (bool)((m >> ((bits >> (8 * j)) & 63u)) & 1ull); };
    // f and the code are read on planes z0-2 .. z1+1, x on z0-3 .. z1+2
    auto fplane = [&](int k) { return k >= z0 - 2 && k <= z1 + 1 && k < nz; };
    struct Regs {
        T x[XR];
        T f[QR];
        uint8_t d[QR];
    };
    // global -> registers for plane k = z0 - 3 + pi
    auto fetch = [&](Regs &r, int k, int pi) {
        const bool kin = k >= 0 && k < nz && k <= z1 + 2;
        const unsigned long long m = kin ? L.m[pi] : 0ull;
        const size_t base = (size_t)min(max(k, 0), nz - 1) * plane;
        const __amdgpu_buffer_rsrc_t rx = rsrc(xin ? xin + base : f + base, xin ? pbytes : 0);
        const __amdgpu_buffer_rsrc_t rf = rsrc(f + base, pbytes);
        const __amdgpu_buffer_rsrc_t rc = rsrc(code + base, (int)plane);
#pragma unroll
        for (int q = 0; q < XR; q++) r.x[q] = bload<T>(rx, mbit(m, q) ? xoff[q] : OFF_NONE);
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const bool p = fplane(k) && qoff[q] >= 0 && mbit(m, XR + q);
            r.f[q] = bload<T>(rf, p ? qoff[q] : OFF_NONE);
            r.d[q] = bload<uint8_t>(rc, p ? qoff[q] >> TSH : OFF_NONE);
        }
    };
    // ring slots from a plane's position j = k - z0 (j >= -3), compile-time
    // in the unrolled march
    auto xslot = [](int j) { return (j + 3 * XS) % XS; };
    auto fslot = [](int j) { return (j + 3 * FS) % FS; };
    auto commit = [&](const Regs &r, int j) {
        T *dx = sx[xslot(j)];
        T *df = sf[fslot(j)];
        uint8_t *dd = sd[fslot(j)];
#pragma unroll
        for (int q = 0; q < XR; q++)
            if (tid + q * NT < PN) dx[tid + q * NT] = r.x[q];
#pragma unroll
        for (int q = 0; q < QR; q++)
            if (tid + q * NT < QN) {
                df[tid + q * NT] = r.f[q];
                dd[tid + q * NT] = r.d[q];
            }
    };
    // relax colour `col` of plane z0 + j on [lo, PX-lo) x [lo, PY-lo), at most
    // one cell per thread (the code is 0 on inactive and out-of-box cells)
    auto relax = [&](int j, int col, int lo) {
        const int k = z0 + j;
        if (k < 0 || k >= nz) return;
        T *c = sx[xslot(j)];
        const T *dn = sx[xslot(j - 1)];
        const T *up = sx[xslot(j + 1)];
        const T *fq = sf[fslot(j)];
        const uint8_t *dq = sd[fslot(j)];
        const int half = (PX - 2 * lo) >> 1;
        const int rows = PY - 2 * lo;
        static_assert(((PX - 2) >> 1) * (PY - 2) <= NT, "one red cell per thread");
        const int e = tid;
        if (e >= half * rows) return;
        const int v = lo + e / half;
        const int u = lo + ((col + gy0 + v + k + gx0 + lo) & 1) + 2 * (e % half);
        const int qq = (v - 1) * QX + (u - 1);
        const int ci = (int)dq[qq];
        if (ci == 0) return;
        const int q = v * PX + u;
        const T s = (c[q - 1] + c[q + 1]) + (c[q - PX] + c[q + PX]) + (dn[q] + up[q]);
        c[q] = rb::div_small<T>(s - h2 * fq[qq], T(ci), L.rcp[ci]);
    };

    // Thread (tu, tv) owns tile cell (x0 + tu, y0 + tv); a wave holds two
    // tile rows, so the lane exchanges over 1 and 32 pair the x and y
    // children of a coarse cell.
    const int tu = tid % BX, tv = tid / BX;
    const int q0 = (tv + H) * PX + (tu + H);
    const int qf = (tv + H - 1) * QX + (tu + H - 1);
    const int ci = sg.x0 + tu, cj = sg.y0 + tv;
    const bool own = ci < nx && cj < ny;
    const int ooff = own ? (cj * nx + ci) * (int)sizeof(T) : OFF_NONE;
    // final x of the last two planes read, the in-plane neighbour sum of the
    // newer one, own f and code of the plane below the last read (A) and of
    // the last read (B), the coarse partial sum
    T xa = T(0), xb = T(0), nb = T(0), fA = T(0), fB = T(0), acc = T(0);
    uint8_t cA = 0, cB = 0;

    // Position p is final: read the own cell and its in-plane neighbours,
    // form the residual of position p - 1 and its share of the restriction,
    // store position p.
    auto final_plane = [&](int p) {
        const T *cp = sx[xslot(p)];
        const T xn = cp[q0];
        const T sn = (cp[q0 - 1] + cp[q0 + 1]) + (cp[q0 - PX] + cp[q0 + PX]);
        if (p >= 1 && p - 1 < zlen) {  // uniform: residual of position p - 1
            T rr = T(0);
            if (cA != 0) rr = ((nb + (xa + xn)) - T((int)cA) * xb) * ih2 - fA;
            T s2 = rr + __shfl_xor(rr, 1);
            s2 += __shfl_xor(s2, 32);
            const int k = z0 + p - 1;
            if ((k & 1) == 0) {
                acc = s2;
            } else {
                acc += s2;
                if ((tu & 1) == 0 && (tv & 1) == 0 && own) {
                    const size_t P = ((size_t)(k >> 1) * cny + (cj >> 1)) * cnx + (ci >> 1);
                    const bool act = L.cf[(p - 1) >> 1][(tv >> 1) * (BX / 2) + (tu >> 1)];
                    fc[P] = act ? -acc / T(8) : T(0);
                }
            }
        }
        if (p >= 0 && p < zlen)  // inactive cells hold 0 in every iterate buffer
            bstore<T>(xn, rsrc(xout + (size_t)(z0 + p) * plane, pbytes), cB != 0 ? ooff : OFF_NONE);
        xa = xb;
        xb = xn;
        nb = sn;
        fA = fB;
        cA = cB;
    };

    // Step st commits position st-3 (positions -3 .. SEGZ+2), relaxes red on
    // position st-4 and black on position st-5, and in its black phase
    // handles the final position st-6 (which that phase does not write).
    // The last step only handles the final position.
    constexpr int NSTEP = SEGZ + 2 * H;
    constexpr int PF = sizeof(T) == 8 ? PF64 : PF32;
    Regs r[PF];
#pragma unroll
    for (int q = 0; q < PF; q++) fetch(r[q], z0 - 3 + q, q);
#pragma unroll
    for (int st = 0; st <= NSTEP; st++) {
        if (st < NSTEP) {
            commit(r[st % PF], st - 3);
            if (st + PF < NSTEP) fetch(r[st % PF], z0 - 3 + st + PF, st + PF);
        }
        __syncthreads();
        if (st == NSTEP) final_plane(st - 6);
        if (st >= 2 && st < NSTEP) relax(st - 4, 0, 1);
        if (st >= 4 && st < NSTEP) {
            __syncthreads();
            relax(st - 5, 1, 2);
            if (st >= 5) final_plane(st - 6);
            fB = sf[fslot(st - 5)][qf];
            cB = sd[fslot(st - 5)][qf];
        }
    }
}

}  // namespace rbr
}  // namespace mg
