// Per-cell and per-column bodies of the residual, restriction, prolongation,
// norm and boundary-folding kernels, shared by the per-level kernels
// (transfer.hip) and the batched phase kernels (batch.hip).
//
// A block of 256 threads covers the TX x TY cross-section of one tile.  The
// stencil bodies give each thread a short z-column and issue every load of the
// column before using any of them (unconditional loads from clamped
// addresses, masked afterwards), so a thread keeps many independent memory
// requests in flight.
#pragma once

#include <type_traits>

#include "mg_core.h"

namespace mg {
namespace tr {

constexpr int NT = TX * TY;  // 256
constexpr int QZ = 4;        // fine planes per thread column
constexpr int NQ = TZ / QZ;  // column blocks per tile

// Work items are dealt to the 8 XCDs round-robin by block id; give each XCD a
// contiguous range of work items so that neighbouring tiles share its L2.
__device__ __forceinline__ int xcd_item(int b, int nb) {
    const int per = nb >> 3;  // nb is a multiple of 8
    return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ int clampi(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

struct TileCoord {
    int i, j, k;
    bool ok;
};

// This thread's cell in plane kk (0 <= kk < TZ) of a tile.
__device__ __forceinline__ TileCoord tile_cell(int tile, int kk, int ntx, int nty, int nx, int ny, int nz) {
    TileCoord t;
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    t.i = tx * TX + (int)(threadIdx.x % TX);
    t.j = ty * TY + (int)(threadIdx.x / TX);
    t.k = tz * TZ + kk;
    t.ok = t.i < nx && t.j < ny && t.k < nz;
    return t;
}

struct Col {
    int i, j, k0;  // first cell of the column
    bool okij;     // (i, j) inside the box
};

// This thread's column of QZ cells in quarter q (0 <= q < NQ) of a tile.
__device__ __forceinline__ Col tile_col(int tile, int q, int ntx, int nty, int nx, int ny) {
    Col c;
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    c.i = tx * TX + (int)(threadIdx.x % TX);
    c.j = ty * TY + (int)(threadIdx.x / TX);
    c.k0 = tz * TZ + q * QZ;
    c.okij = c.i < nx && c.j < ny;
    return c;
}

// Diagonal of the level's operator at cell p, 0 if inactive.
template <typename T, bool FINE>
__device__ __forceinline__ T diag_at(const uint8_t *code, const T *dco, size_t p) {
    if constexpr (FINE) {
        const uint8_t c = code[p];
        return T((int)c);  // CODE_OFF is 0
    } else {
        return dco[p];
    }
}

// Deterministic block sum of one double per thread (fixed lane and wave order);
// the result is valid in thread 0.
__device__ inline double block_sum(double v) {
    __shared__ double ws[NT / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) ws[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < NT / 64; q++) t += ws[q];
    __syncthreads();
    return t;
}

// Residual r = h^-2 (sum_j x_j - d x) - f of NZ cells of a column (Sec. 2
// 7-point Laplacian; the Sec. 3 ghost is folded into d), with the box edge
// treated as x = 0.  dv[q] == 0 marks inactive cells (r = 0).
template <typename T, bool FINE, int NZ = QZ>
__device__ __forceinline__ void column_residual(const T *__restrict__ x, const T *__restrict__ f,
                                                const uint8_t *__restrict__ code, const T *__restrict__ dco,
                                                int i, int j, int k0, bool okij, int nx, int ny, int nz, T ih2,
                                                T (&r)[NZ], T (&dv)[NZ]) {
    const size_t pl = (size_t)nx * ny;
    const int ic = clampi(i, nx - 1), jc = clampi(j, ny - 1);
    const size_t c0 = (size_t)jc * nx + ic;
    const size_t cxm = (size_t)jc * nx + clampi(i - 1, nx - 1), cxp = (size_t)jc * nx + clampi(i + 1, nx - 1);
    const size_t cym = (size_t)clampi(j - 1, ny - 1) * nx + ic, cyp = (size_t)clampi(j + 1, ny - 1) * nx + ic;
    T xs[NZ + 2], xm[NZ], xp[NZ], ym[NZ], yp[NZ], fv[NZ];
    typename std::conditional<FINE, uint8_t, T>::type dr[NZ];
#pragma unroll
    for (int q = 0; q < NZ + 2; q++) xs[q] = x[(size_t)clampi(k0 - 1 + q, nz - 1) * pl + c0];
#pragma unroll
    for (int q = 0; q < NZ; q++) {
        const size_t b = (size_t)clampi(k0 + q, nz - 1) * pl;
        xm[q] = x[b + cxm];
        xp[q] = x[b + cxp];
        ym[q] = x[b + cym];
        yp[q] = x[b + cyp];
        fv[q] = f[b + c0];
        if constexpr (FINE) dr[q] = code[b + c0];
        else dr[q] = dco[b + c0];
    }
    const bool bxm = i > 0, bxp = i < nx - 1, bym = j > 0, byp = j < ny - 1;
#pragma unroll
    for (int q = 0; q < NZ; q++) {
        const int k = k0 + q;
        T d;
        if constexpr (FINE) d = T((int)dr[q]);  // CODE_OFF is 0
        else d = dr[q];
        if (!okij || k >= nz) d = T(0);
        const T zm = k > 0 ? xs[q] : T(0);
        const T zp = k < nz - 1 ? xs[q + 2] : T(0);
        const T s = ((bxm ? xm[q] : T(0)) + (bxp ? xp[q] : T(0))) + ((bym ? ym[q] : T(0)) + (byp ? yp[q] : T(0))) +
                    (zm + zp);
        dv[q] = d;
        r[q] = d != T(0) ? (s - d * xs[q + 1]) * ih2 - fv[q] : T(0);
    }
}

// ---- fold the Dirichlet values into the right-hand side, load the guess ----
// With the boundary on the face between active i and inactive j (theta = 1/2),
// the ghost is 2 g_ij - x_i with g_ij = (B_i + B_j)/2 (Sec. 3, Fig. "ghost"),
// so the known part B_i + B_j moves to the right-hand side.  Active cells are
// never on the box edge (validated), so their six neighbours exist.
__device__ __forceinline__ void fold_cell(const TileCoord &t, int nx, int ny, double ih2,
                                          const uint8_t *__restrict__ code, const double *__restrict__ rho,
                                          const double *__restrict__ B, const double *__restrict__ phi,
                                          double *__restrict__ f, double *__restrict__ x) {
    if (!t.ok) return;
    const size_t pl = (size_t)nx * ny;
    const size_t p = (size_t)t.k * pl + (size_t)t.j * nx + t.i;
    const uint8_t c = code[p];
    if (c == CODE_OFF) {
        f[p] = 0.0;
        if (x) x[p] = 0.0;
        return;
    }
    double fv = rho[p];
    if (B && c > 6) {  // some face neighbour is inactive
        const double bi = B[p];
        double g = 0.0;
        if (code[p - 1] == CODE_OFF) g += bi + B[p - 1];
        if (code[p + 1] == CODE_OFF) g += bi + B[p + 1];
        if (code[p - nx] == CODE_OFF) g += bi + B[p - nx];
        if (code[p + nx] == CODE_OFF) g += bi + B[p + nx];
        if (code[p - pl] == CODE_OFF) g += bi + B[p - pl];
        if (code[p + pl] == CODE_OFF) g += bi + B[p + pl];
        fv -= ih2 * g;
    }
    f[p] = fv;
    if (x) x[p] = phi ? phi[p] : 0.0;
}

__device__ __forceinline__ void store_cell(const TileCoord &t, int nx, int ny, const uint8_t *__restrict__ code,
                                           const double *__restrict__ x, double *__restrict__ phi) {
    if (!t.ok) return;
    const size_t p = (size_t)t.k * nx * ny + (size_t)t.j * nx + t.i;
    if (code[p] != CODE_OFF) phi[p] = x[p];
}

// ---- residual norm of a column: sum over its active cells of (L x - f)^2 ----
// Optionally writes r32 = f - L x in float (mixed-precision inner right-hand
// side).  Returns this thread's partial sum.
template <bool FINE, bool HASX, bool W32>
__device__ __forceinline__ double resnorm_col(const Col &c, int nx, int ny, int nz, double ih2,
                                              const uint8_t *__restrict__ code, const double *__restrict__ dco,
                                              const double *__restrict__ x, const double *__restrict__ f,
                                              float *__restrict__ r32) {
    double r[QZ], dv[QZ];
    if constexpr (HASX) {
        column_residual<double, FINE>(x, f, code, dco, c.i, c.j, c.k0, c.okij, nx, ny, nz, ih2, r, dv);
    } else {
        const size_t pl = (size_t)nx * ny;
        const size_t c0 = (size_t)clampi(c.j, ny - 1) * nx + clampi(c.i, nx - 1);
#pragma unroll
        for (int q = 0; q < QZ; q++) {
            const size_t b = (size_t)clampi(c.k0 + q, nz - 1) * pl;
            const double fv = f[b + c0];
            const double d = diag_at<double, FINE>(code, dco, b + c0);
            r[q] = (c.okij && c.k0 + q < nz && d != 0.0) ? -fv : 0.0;
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < QZ; q++) acc += r[q] * r[q];
    if constexpr (W32) {
        const size_t pl = (size_t)nx * ny;
#pragma unroll
        for (int q = 0; q < QZ; q++)
            if (c.okij && c.k0 + q < nz) r32[(size_t)(c.k0 + q) * pl + (size_t)c.j * nx + c.i] = (float)(-r[q]);
    }
    return acc;
}

// ---- R1 restriction of the residual (Sec. 2 steps 2-5) ----
// Coarse active cell t gets f_c = -(1/8) sum over its active children of
// r = L x - f; the coarse problem is Delta_c dPhi = -r_c.  The 2 x 2 x 2
// children and their face neighbours are loaded together.
template <typename T, bool FINE>
__device__ __forceinline__ void restrict_cell(const TileCoord &t, int cnx, int cny, const T *__restrict__ cd, int nx,
                                              int ny, int nz, T ih2, const uint8_t *__restrict__ code,
                                              const T *__restrict__ dco, const T *__restrict__ x,
                                              const T *__restrict__ f, T *__restrict__ fc) {
    if (!t.ok) return;
    const size_t P = (size_t)t.k * cnx * cny + (size_t)t.j * cnx + t.i;
    const T cdv = cd[P];
    const int i0 = 2 * t.i, j0 = 2 * t.j, k0 = 2 * t.k;
    // r[b][a][e]: child (i0 + a, j0 + b, k0 + e); inactive children give 0
    T r[2][2][2], d[2][2][2];
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
        for (int a = 0; a < 2; a++)
            column_residual<T, FINE, 2>(x, f, code, dco, i0 + a, j0 + b, k0, true, nx, ny, nz, ih2, r[b][a], d[b][a]);
    T s = T(0);
#pragma unroll
    for (int c = 0; c < 8; c++) s += r[(c >> 1) & 1][c & 1][c >> 2];  // children in x, y, z order
    fc[P] = cdv != T(0) ? -s / T(8) : T(0);
}

// ---- P2 prolongation and correction of a column (Sec. 2 steps 6-7) ----
// Along each axis the fine centre lies a quarter coarse cell from its parent
// towards the side of its child offset: weights 3/4 (parent) and 1/4 (the
// coarse neighbour on that side); coarse values off the coarse domain are 0.
template <typename T, bool FINE>
__device__ __forceinline__ void prolong_col(const Col &c, int nx, int ny, int nz, const uint8_t *__restrict__ code,
                                            const T *__restrict__ dco, const T *__restrict__ xc, int cnx, int cny,
                                            int cnz, T *__restrict__ x) {
    if (!c.okij) return;
    const size_t pl = (size_t)nx * ny, cpl = (size_t)cnx * cny;
    const int I = c.i >> 1, J = c.j >> 1, K0 = c.k0 >> 1;  // k0 is even
    const int sx = (c.i & 1) ? 1 : -1, sy = (c.j & 1) ? 1 : -1;
    // coarse columns: (I, J), (I+sx, J), (I, J+sy), (I+sx, J+sy); planes K0-1 .. K0+2
    const int ci[2] = {I, I + sx}, cj[2] = {J, J + sy};
    T cv[2][2][4];
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
        for (int a = 0; a < 2; a++) {
            const bool okc = ci[a] >= 0 && ci[a] < cnx && cj[b] >= 0 && cj[b] < cny;
            const size_t cc = (size_t)clampi(cj[b], cny - 1) * cnx + clampi(ci[a], cnx - 1);
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int K = K0 - 1 + q;
                const T v = xc[(size_t)clampi(K, cnz - 1) * cpl + cc];
                cv[b][a][q] = (okc && K >= 0 && K < cnz) ? v : T(0);
            }
        }
    T xv[QZ];
    typename std::conditional<FINE, uint8_t, T>::type dr[QZ];
    const size_t c0 = (size_t)c.j * nx + c.i;
#pragma unroll
    for (int q = 0; q < QZ; q++) {
        const size_t b = (size_t)clampi(c.k0 + q, nz - 1) * pl;
        xv[q] = x[b + c0];
        if constexpr (FINE) dr[q] = code[b + c0];
        else dr[q] = dco[b + c0];
    }
    const T w4[2] = {T(0.75), T(0.25)};
#pragma unroll
    for (int q = 0; q < QZ; q++) {
        const int k = c.k0 + q;
        bool act;
        if constexpr (FINE) act = dr[q] != CODE_OFF;
        else act = dr[q] != T(0);
        if (k >= nz || !act) continue;
        // parent plane index in cv: K - (K0 - 1); neighbour plane on the side of the child offset
        const int pk = (k >> 1) - (K0 - 1);
        const int nk = pk + ((k & 1) ? 1 : -1);
        T s = T(0);
#pragma unroll
        for (int cz = 0; cz < 2; cz++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int a = 0; a < 2; a++) s += w4[a] * w4[b] * w4[cz] * cv[b][a][cz ? nk : pk];
        x[(size_t)k * pl + c0] = xv[q] + s;
    }
}

}  // namespace tr
}  // namespace mg
