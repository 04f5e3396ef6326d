// Residual, restriction, prolongation, norms and boundary folding.
//
// Thread-per-cell kernels over active tiles: a block of 256 threads covers a
// TX x TY column of one tile and walks its TZ planes.  Neighbour values come
// from the L1/L2 caches.
#include <type_traits>

#include "mg_core.h"

namespace mg {

namespace {

constexpr int NT = TX * TY;  // 256

__device__ __forceinline__ int xcd_item(int b, int nb) {
    const int per = nb >> 3;
    return (b & 7) * per + (b >> 3);
}

inline unsigned grid8(int items) { return (unsigned)(((items + 7) / 8) * 8); }
inline unsigned gridt(int ntiles) { return grid8(ntiles * TZ); }


struct TileCoord {
    int i, j, k;
    bool ok;
};

// One block per (active tile, plane of the tile): w = item * TZ + plane.
// Returns false when the block has no tile (padding of the grid to 8).
__device__ __forceinline__ bool tile_coord(const int *tiles, int ntiles, int ntx, int nty, int nx, int ny, int nz,
                                           TileCoord &t, int &w) {
    w = xcd_item(blockIdx.x, gridDim.x);
    const int item = w / TZ;
    if (item >= ntiles) return false;
    const int tile = tiles[item];
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    t.i = tx * TX + (int)(threadIdx.x % TX);
    t.j = ty * TY + (int)(threadIdx.x / TX);
    t.k = tz * TZ + w % TZ;
    t.ok = t.i < nx && t.j < ny && t.k < nz;
    return true;
}

// Diagonal of the level's operator at cell p, 0 if inactive.
template <typename T, bool FINE>
__device__ __forceinline__ T diag_at(const uint8_t *code, const T *dco, size_t p) {
    if constexpr (FINE) {
        const uint8_t c = code[p];
        return c == CODE_OFF ? T(0) : T(12 - (int)c);
    } else {
        return dco[p];
    }
}

// h^2 (L x)_i = sum of the six neighbours - d_i x_i, with x = 0 off the domain
// and out of the box (Sec. 2 7-point Laplacian with the Sec. 3 ghost folded
// into d_i).
template <typename T>
__device__ __forceinline__ T nsum(const T *x, size_t p, int i, int j, int k, int nx, int ny, int nz) {
    const size_t pl = (size_t)nx * ny;
    const T xm = i > 0 ? x[p - 1] : T(0);
    const T xp = i < nx - 1 ? x[p + 1] : T(0);
    const T ym = j > 0 ? x[p - nx] : T(0);
    const T yp = j < ny - 1 ? x[p + nx] : T(0);
    const T zm = k > 0 ? x[p - pl] : T(0);
    const T zp = k < nz - 1 ? x[p + pl] : T(0);
    return (xm + xp) + (ym + yp) + (zm + zp);
}

// Deterministic block sum of one double per thread (fixed lane and wave order).
__device__ double block_sum(double v) {
    __shared__ double ws[NT / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) ws[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < NT / 64; q++) t += ws[q];
    return t;
}

// ---- fold the Dirichlet values into the right-hand side, load the guess ----
// With the boundary on the face between active i and inactive j (theta = 1/2),
// the ghost is 2 g_ij - x_i with g_ij = (B_i + B_j)/2 (Sec. 3, Fig. "ghost"),
// so the known part B_i + B_j moves to the right-hand side.
__global__ __launch_bounds__(NT) void k_fold(const int *__restrict__ tiles, int ntiles, int ntx, int nty, int nx,
                                             int ny, int nz, double ih2, const uint8_t *__restrict__ code,
                                             const double *__restrict__ rho, const double *__restrict__ B,
                                             const double *__restrict__ phi, double *__restrict__ f,
                                             double *__restrict__ x) {
    TileCoord t;
    int w;
    if (!tile_coord(tiles, ntiles, ntx, nty, nx, ny, nz, t, w) || !t.ok) return;
    const size_t pl = (size_t)nx * ny;
    {
        const int k = t.k;
        const size_t p = (size_t)k * pl + (size_t)t.j * nx + t.i;
        const uint8_t c = code[p];
        if (c == CODE_OFF) {
            f[p] = 0.0;
            if (x) x[p] = 0.0;
            return;
        }
        double fv = rho[p];
        if (B && c < 6) {
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
}

__global__ __launch_bounds__(NT) void k_store(const int *__restrict__ tiles, int ntiles, int ntx, int nty, int nx,
                                              int ny, int nz, const uint8_t *__restrict__ code,
                                              const double *__restrict__ x, double *__restrict__ phi) {
    TileCoord t;
    int w;
    if (!tile_coord(tiles, ntiles, ntx, nty, nx, ny, nz, t, w) || !t.ok) return;
    const size_t pl = (size_t)nx * ny;
    {
        const int k = t.k;
        const size_t p = (size_t)k * pl + (size_t)t.j * nx + t.i;
        if (code[p] != CODE_OFF) phi[p] = x[p];
    }
}

template <bool FINE>
__global__ __launch_bounds__(NT) void k_copy_masked(const int *__restrict__ tiles, int ntiles, int ntx, int nty,
                                                    int nx, int ny, int nz, const uint8_t *__restrict__ code,
                                                    const double *__restrict__ dco, const double *__restrict__ src,
                                                    double *__restrict__ dst) {
    TileCoord t;
    int w;
    if (!tile_coord(tiles, ntiles, ntx, nty, nx, ny, nz, t, w) || !t.ok) return;
    const size_t pl = (size_t)nx * ny;
    {
        const int k = t.k;
        const size_t p = (size_t)k * pl + (size_t)t.j * nx + t.i;
        dst[p] = diag_at<double, FINE>(code, dco, p) != 0.0 ? src[p] : 0.0;
    }
}

// ---- column loads ----------------------------------------------------------
// The stencil kernels below give each thread a short z-column of QZ cells and
// issue every load of the column before using any of them (unconditional
// loads from clamped addresses, masked afterwards), so a thread keeps a dozen
// or more independent memory requests in flight.
constexpr int QZ = 4;            // fine planes per thread column
constexpr int NQ = TZ / QZ;      // column blocks per tile
inline unsigned gridc(int ntiles) { return grid8(ntiles * NQ); }

struct Col {
    int i, j, k0;        // first cell of the column
    bool okij;           // (i, j) inside the box
    int w;               // block work index
};

__device__ __forceinline__ bool col_coord(const int *tiles, int ntiles, int ntx, int nty, int nx, int ny, Col &c) {
    c.w = xcd_item(blockIdx.x, gridDim.x);
    const int item = c.w / NQ;
    if (item >= ntiles) return false;
    const int tile = tiles[item];
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    c.i = tx * TX + (int)(threadIdx.x % TX);
    c.j = ty * TY + (int)(threadIdx.x / TX);
    c.k0 = tz * TZ + (c.w % NQ) * QZ;
    c.okij = c.i < nx && c.j < ny;
    return true;
}

__device__ __forceinline__ int clampi(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }

// Residual r = h^-2 (sum_j x_j - d x) - f of the QZ cells of a column, with
// the box edge treated as x = 0.  d[q] == 0 marks inactive cells (r = 0).
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
        if constexpr (FINE) d = dr[q] == CODE_OFF ? T(0) : T(12 - (int)dr[q]);
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

// ---- residual norm: sum over active cells of (L x - f)^2 ----
// Optionally writes r32 = f - L x in float (mixed-precision inner right-hand
// side).  Partial sums per block, then a fixed-order total.
template <bool FINE, bool HASX, bool W32>
__global__ __launch_bounds__(NT) void k_resnorm(const int *__restrict__ tiles, int ntiles, int ntx, int nty, int nx,
                                                int ny, int nz, double ih2, const uint8_t *__restrict__ code,
                                                const double *__restrict__ dco, const double *__restrict__ x,
                                                const double *__restrict__ f, double *__restrict__ part,
                                                float *__restrict__ r32) {
    Col c;
    if (!col_coord(tiles, ntiles, ntx, nty, nx, ny, c)) return;  // uniform per block
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
    const double s = block_sum(acc);
    if (threadIdx.x == 0) part[c.w] = s;
}

__global__ __launch_bounds__(1024) void k_finalize(const double *__restrict__ part, int n, double *__restrict__ out,
                                                   int slot) {
    __shared__ double sm[1024];
    double v = 0.0;
    for (int q = threadIdx.x; q < n; q += 1024) v += part[q];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[slot] = sm[0];
}

template <bool FINE>
__global__ __launch_bounds__(NT) void k_residual(const int *__restrict__ tiles, int ntiles, int ntx, int nty, int nx,
                                                 int ny, int nz, double ih2, const uint8_t *__restrict__ code,
                                                 const double *__restrict__ dco, const double *__restrict__ x,
                                                 const double *__restrict__ f, double *__restrict__ r) {
    Col c;
    if (!col_coord(tiles, ntiles, ntx, nty, nx, ny, c)) return;
    double rr[QZ], dv[QZ];
    column_residual<double, FINE>(x, f, code, dco, c.i, c.j, c.k0, c.okij, nx, ny, nz, ih2, rr, dv);
    if (!c.okij) return;
    const size_t pl = (size_t)nx * ny;
#pragma unroll
    for (int q = 0; q < QZ; q++)
        if (c.k0 + q < nz) r[(size_t)(c.k0 + q) * pl + (size_t)c.j * nx + c.i] = rr[q];
}

// ---- R1 restriction of the residual (Sec. 2 steps 2-5) ----
// Coarse active cell I gets f_c = -(1/8) sum over its active children of
// r = L x - f; the coarse problem is Delta_c dPhi = -r_c.  One thread per
// coarse cell; the 2 x 2 x 2 children and their face neighbours are loaded
// together.
template <typename T, bool FINE>
__global__ __launch_bounds__(NT) void k_restrict(const int *__restrict__ ctiles, int ntiles, int cntx, int cnty,
                                                 int cnx, int cny, int cnz, const T *__restrict__ cd, int nx, int ny,
                                                 int nz, T ih2, const uint8_t *__restrict__ code,
                                                 const T *__restrict__ dco, const T *__restrict__ x,
                                                 const T *__restrict__ f, T *__restrict__ fc) {
    TileCoord t;
    int w;
    if (!tile_coord(ctiles, ntiles, cntx, cnty, cnx, cny, cnz, t, w) || !t.ok) return;
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

// ---- P2 prolongation and correction (Sec. 2 steps 6-7) ----
// Along each axis the fine centre lies a quarter coarse cell from its parent
// towards the side of its child offset: weights 3/4 (parent) and 1/4 (the
// coarse neighbour on that side); coarse values off the coarse domain are 0.
template <typename T, bool FINE>
__global__ __launch_bounds__(NT) void k_prolong(const int *__restrict__ tiles, int ntiles, int ntx, int nty, int nx,
                                                int ny, int nz, const uint8_t *__restrict__ code,
                                                const T *__restrict__ dco, const T *__restrict__ xc, int cnx, int cny,
                                                int cnz, T *__restrict__ x) {
    Col c;
    if (!col_coord(tiles, ntiles, ntx, nty, nx, ny, c) || !c.okij) return;
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

template <typename T>
__global__ __launch_bounds__(NT) void k_zero_tiles(const int *__restrict__ tiles, int ntiles, int ntx, int nty, int nx,
                                                   int ny, int nz, T *__restrict__ x) {
    TileCoord t;
    int w;
    if (!tile_coord(tiles, ntiles, ntx, nty, nx, ny, nz, t, w) || !t.ok) return;
    x[(size_t)t.k * nx * ny + (size_t)t.j * nx + t.i] = T(0);
}

__global__ __launch_bounds__(NT) void k_axpy32(const int *__restrict__ tiles, int ntiles, int ntx, int nty, int nx,
                                               int ny, int nz, const uint8_t *__restrict__ code,
                                               const float *__restrict__ e, double *__restrict__ x) {
    TileCoord t;
    int w;
    if (!tile_coord(tiles, ntiles, ntx, nty, nx, ny, nz, t, w) || !t.ok) return;
    const size_t p = (size_t)t.k * nx * ny + (size_t)t.j * nx + t.i;
    if (code[p] != CODE_OFF) x[p] += (double)e[p];
}

}  // namespace

void launch_fold(const Level &L, const OrderData &od, const double *rho, const double *B, const double *phi,
                 double *f, double *x, hipStream_t s) {
    if (!od.ntiles) return;
    k_fold<<<gridt(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz, 1.0 / (L.h * L.h),
                                           L.code, rho, B, phi, f, x);
}

void launch_store(const Level &L, const OrderData &od, const double *x, double *phi, hipStream_t s) {
    if (!od.ntiles) return;
    k_store<<<gridt(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz, L.code, x, phi);
}

void launch_copy_masked(const Level &L, int level, const OrderData &od, const double *src, double *dst,
                        hipStream_t s) {
    if (!od.ntiles) return;
    if (level == 0)
        k_copy_masked<true><<<gridt(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz,
                                                            L.code, nullptr, src, dst);
    else
        k_copy_masked<false><<<gridt(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz,
                                                             nullptr, od.d, src, dst);
}

void launch_resnorm(const Level &L, int level, const OrderData &od, const double *x, const double *f, double *part,
                    double *out, int slot, hipStream_t s) {
    const double ih2 = 1.0 / (L.h * L.h);
    const unsigned g = gridc(od.ntiles);
    if (od.ntiles) {
        if (level == 0) {
            if (x)
                k_resnorm<true, true, false><<<g, NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz, ih2,
                                                              L.code, nullptr, x, f, part, nullptr);
            else
                k_resnorm<true, false, false><<<g, NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz,
                                                               ih2, L.code, nullptr, x, f, part, nullptr);
        } else {
            k_resnorm<false, true, false><<<g, NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz, ih2,
                                                           nullptr, od.d, x, f, part, nullptr);
        }
    }
    k_finalize<<<1, 1024, 0, s>>>(part, od.ntiles * NQ, out, slot);
}

void launch_resnorm32(const Level &L, const OrderData &od, const double *x, const double *f, float *r32, double *part,
                      double *out, int slot, hipStream_t s) {
    const double ih2 = 1.0 / (L.h * L.h);
    if (od.ntiles)
        k_resnorm<true, true, true><<<gridc(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny,
                                                                    L.nz, ih2, L.code, nullptr, x, f, part, r32);
    k_finalize<<<1, 1024, 0, s>>>(part, od.ntiles * NQ, out, slot);
}

void launch_residual(const Level &L, int level, const OrderData &od, const double *x, const double *f, double *r,
                     hipStream_t s) {
    if (!od.ntiles) return;
    const double ih2 = 1.0 / (L.h * L.h);
    if (level == 0)
        k_residual<true><<<gridc(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz, ih2,
                                                         L.code, nullptr, x, f, r);
    else
        k_residual<false><<<gridc(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz, ih2,
                                                          nullptr, od.d, x, f, r);
}

void launch_restrict(const Level &L, const Level &C, int level, int order, const double *x, const double *f,
                     double *fc, hipStream_t s) {
    const OrderData &co = C.od[order];
    if (!co.ntiles) return;
    const double ih2 = 1.0 / (L.h * L.h);
    if (level == 0)
        k_restrict<double, true><<<gridt(co.ntiles), NT, 0, s>>>(co.tiles, co.ntiles, C.ntx, C.nty, C.nx, C.ny, C.nz,
                                                                 co.d, L.nx, L.ny, L.nz, ih2, L.code, nullptr, x, f,
                                                                 fc);
    else
        k_restrict<double, false><<<gridt(co.ntiles), NT, 0, s>>>(co.tiles, co.ntiles, C.ntx, C.nty, C.nx, C.ny,
                                                                  C.nz, co.d, L.nx, L.ny, L.nz, ih2, nullptr,
                                                                  L.od[order].d, x, f, fc);
}

void launch_restrict32(const Level &L, const Level &C, int level, int order, const float *x, const float *f,
                       float *fc, hipStream_t s) {
    const OrderData &co = C.od[order];
    if (!co.ntiles) return;
    const float ih2 = (float)(1.0 / (L.h * L.h));
    if (level == 0)
        k_restrict<float, true><<<gridt(co.ntiles), NT, 0, s>>>(co.tiles, co.ntiles, C.ntx, C.nty, C.nx, C.ny, C.nz,
                                                                co.d32, L.nx, L.ny, L.nz, ih2, L.code, nullptr, x, f,
                                                                fc);
    else
        k_restrict<float, false><<<gridt(co.ntiles), NT, 0, s>>>(co.tiles, co.ntiles, C.ntx, C.nty, C.nx, C.ny, C.nz,
                                                                 co.d32, L.nx, L.ny, L.nz, ih2, nullptr,
                                                                 L.od[order].d32, x, f, fc);
}

void launch_prolong(const Level &L, const Level &C, int level, int order, const double *xc, double *x,
                    hipStream_t s) {
    const OrderData &od = L.od[level == 0 ? 2 : order];
    if (!od.ntiles) return;
    if (level == 0)
        k_prolong<double, true><<<gridc(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz,
                                                                L.code, nullptr, xc, C.nx, C.ny, C.nz, x);
    else
        k_prolong<double, false><<<gridc(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz,
                                                                 nullptr, od.d, xc, C.nx, C.ny, C.nz, x);
}

void launch_prolong32(const Level &L, const Level &C, int level, int order, const float *xc, float *x,
                      hipStream_t s) {
    const OrderData &od = L.od[level == 0 ? 2 : order];
    if (!od.ntiles) return;
    if (level == 0)
        k_prolong<float, true><<<gridc(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz,
                                                               L.code, nullptr, xc, C.nx, C.ny, C.nz, x);
    else
        k_prolong<float, false><<<gridc(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz,
                                                                nullptr, od.d32, xc, C.nx, C.ny, C.nz, x);
}

void launch_zero_tiles(const Level &L, const OrderData &od, double *x, hipStream_t s) {
    if (!od.ntiles) return;
    k_zero_tiles<double><<<gridt(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz, x);
}

void launch_zero_tiles32(const Level &L, const OrderData &od, float *x, hipStream_t s) {
    if (!od.ntiles) return;
    k_zero_tiles<float><<<gridt(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz, x);
}

void launch_axpy32(const Level &L, const OrderData &od, const float *e, double *x, hipStream_t s) {
    if (!od.ntiles) return;
    k_axpy32<<<gridt(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz, L.code, e, x);
}

}  // namespace mg
