// Residual, restriction, prolongation, norms and boundary folding: kernels
// over the active tiles of one level (bodies in transfer_core.h).
#include "march_core.h"

namespace mg {

namespace {

using namespace tr;

inline unsigned grid8(int items) { return (unsigned)(((items + 7) / 8) * 8); }
inline unsigned gridt(int ntiles) { return grid8(ntiles * TZ); }  // one block per (tile, plane)
inline unsigned gridc(int ntiles) { return grid8(ntiles * NQ); }  // one block per (tile, quarter)

// Block work index w -> (tile, sub-block); false for grid padding and when
// the solve loop's halt flag is set.
__device__ __forceinline__ bool block_tile(const int *tiles, int ntiles, int per, int &tile, int &sub, int &w,
                                           const int *halt = nullptr) {
    w = xcd_item(blockIdx.x, gridDim.x);
    const int item = w / per;
    if (item >= ntiles || (halt && *halt)) return false;
    tile = tiles[item];
    sub = w % per;
    return true;
}

__global__ __launch_bounds__(NT) void k_fold(const int *__restrict__ tiles, int ntiles, int ntx, int nty, int nx,
                                             int ny, int nz, double ih2, const uint8_t *__restrict__ code,
                                             const double *__restrict__ rho, const double *__restrict__ B,
                                             const double *__restrict__ phi, double *__restrict__ f,
                                             double *__restrict__ x) {
    int tile, kk, w;
    if (!block_tile(tiles, ntiles, TZ, tile, kk, w)) return;
    fold_cell(tile_cell(tile, kk, ntx, nty, nx, ny, nz), nx, ny, ih2, code, rho, B, phi, f, x);
}

__global__ __launch_bounds__(NT) void k_store(const int *__restrict__ tiles, int ntiles, int ntx, int nty, int nx,
                                              int ny, int nz, const uint8_t *__restrict__ code,
                                              const double *__restrict__ x, double *__restrict__ phi) {
    int tile, kk, w;
    if (!block_tile(tiles, ntiles, TZ, tile, kk, w)) return;
    store_cell(tile_cell(tile, kk, ntx, nty, nx, ny, nz), nx, ny, code, x, phi);
}

template <bool FINE>
__global__ __launch_bounds__(NT) void k_copy_masked(const int *__restrict__ tiles, int ntiles, int ntx, int nty,
                                                    int nx, int ny, int nz, const uint8_t *__restrict__ code,
                                                    const double *__restrict__ dco, const double *__restrict__ src,
                                                    double *__restrict__ dst) {
    int tile, kk, w;
    if (!block_tile(tiles, ntiles, TZ, tile, kk, w)) return;
    const TileCoord t = tile_cell(tile, kk, ntx, nty, nx, ny, nz);
    if (!t.ok) return;
    const size_t p = (size_t)t.k * nx * ny + (size_t)t.j * nx + t.i;
    dst[p] = diag_at<double, FINE>(code, dco, p) != 0.0 ? src[p] : 0.0;
}

// Sum of squares of the residual: partial sums per block (tile quarter), then
// a fixed-order total in k_finalize.
template <bool FINE, bool HASX, bool W32>
__global__ __launch_bounds__(NT) void k_resnorm(const int *__restrict__ tiles, int ntiles, int ntx, int nty, int nx,
                                                int ny, int nz, double ih2, const uint8_t *__restrict__ code,
                                                const double *__restrict__ dco, const double *__restrict__ x,
                                                const double *__restrict__ f, double *__restrict__ part,
                                                float *__restrict__ r32) {
    int tile, q, w;
    if (!block_tile(tiles, ntiles, NQ, tile, q, w)) return;  // uniform per block
    const double acc = resnorm_col<FINE, HASX, W32>(tile_col(tile, q, ntx, nty, nx, ny), nx, ny, nz, ih2, code, dco,
                                                    x, f, r32);
    const double s = block_sum(acc);
    if (threadIdx.x == 0) part[w] = s;
}

__global__ __launch_bounds__(1024) void k_finalize(const double *__restrict__ part, int n, double *__restrict__ out,
                                                   int slot, StopTest *__restrict__ stop, int *__restrict__ halt,
                                                   double *__restrict__ host_out = nullptr) {
    __shared__ double sm[1024];
    if (halt && *halt) return;
    double v = 0.0;
    for (int q = threadIdx.x; q < n; q += 1024) v += part[q];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[slot] = sm[0];
        if (host_out)  // coherent host memory: a system-scope store reaches it directly
            __hip_atomic_store(reinterpret_cast<unsigned long long *>(host_out), __double_as_longlong(sm[0]),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        if (stop) {
            const double r = sqrt(sm[0]);
            const bool h = !(r > stop->thresh) || !isfinite(r) || (stop->check_switch && r / stop->rprev > stop->eta);
            stop->rprev = r;
            *halt = h ? 1 : 0;
        }
    }
}

__global__ void k_set_halt(int *__restrict__ halt, int v) { *halt = v; }

__global__ void k_set_stop(StopTest *__restrict__ st, double thresh, double rprev, double eta, int check_switch) {
    st->thresh = thresh;
    st->rprev = rprev;
    st->eta = eta;
    st->check_switch = check_switch;
    st->pad = 0;
}

template <bool FINE>
__global__ __launch_bounds__(NT) void k_residual(const int *__restrict__ tiles, int ntiles, int ntx, int nty, int nx,
                                                 int ny, int nz, double ih2, const uint8_t *__restrict__ code,
                                                 const double *__restrict__ dco, const double *__restrict__ x,
                                                 const double *__restrict__ f, double *__restrict__ r) {
    int tile, q, w;
    if (!block_tile(tiles, ntiles, NQ, tile, q, w)) return;
    const Col c = tile_col(tile, q, ntx, nty, nx, ny);
    double rr[QZ], dv[QZ];
    column_residual<double, FINE>(x, f, code, dco, c.i, c.j, c.k0, c.okij, nx, ny, nz, ih2, rr, dv);
    if (!c.okij) return;
    const size_t pl = (size_t)nx * ny;
#pragma unroll
    for (int k = 0; k < QZ; k++)
        if (c.k0 + k < nz) r[(size_t)(c.k0 + k) * pl + (size_t)c.j * nx + c.i] = rr[k];
}

template <typename T, bool FINE>
__global__ __launch_bounds__(NT) void k_restrict(const int *__restrict__ ctiles, int ntiles, int cntx, int cnty,
                                                 int cnx, int cny, int cnz, const T *__restrict__ cd, int nx, int ny,
                                                 int nz, T ih2, const uint8_t *__restrict__ code,
                                                 const T *__restrict__ dco, const T *__restrict__ x,
                                                 const T *__restrict__ f, T *__restrict__ fc,
                                                 const int *__restrict__ halt) {
    int tile, kk, w;
    if (!block_tile(ctiles, ntiles, TZ, tile, kk, w, halt)) return;
    restrict_cell<T, FINE>(tile_cell(tile, kk, cntx, cnty, cnx, cny, cnz), cnx, cny, cd, nx, ny, nz, ih2, code, dco,
                           x, f, fc);
}

// Eight blocks per CU put the 2048 finest items of 256^3 in one round (the
// update-and-residual mode keeps seven: eight would spill).
template <typename T, int SEGZ, int MODE>
__global__ __launch_bounds__(NT, MODE == RM_AXPY32 ? 7 : 8) void k_residual_march(
    const T *__restrict__ x, const T *__restrict__ f, const uint8_t *__restrict__ code, int nx, int ny, int nz, T ih2,
    const Seg *__restrict__ segs, const unsigned long long *__restrict__ pm, int nsegs, const T *__restrict__ cd,
    int cnx, int cny, T *__restrict__ fc, double *__restrict__ part, float *__restrict__ r32,
    const float *__restrict__ ecor, T *__restrict__ xo, const int *__restrict__ halt) {
    __shared__ ResLds<T> lds;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= nsegs || (halt && *halt)) return;
    const double sq = residual_item<T, SEGZ, MODE>(lds, x, f, code, nx, ny, nz, ih2, segs[item],
                                                   pm + (size_t)item * (SEGZ + 4), cd, cnx, cny, fc, r32, ecor, xo);
    if constexpr (MODE != RM_RESTRICT) {
        const double t = block_sum(sq);
        if (threadIdx.x == 0) part[item] = t;
    }
}

// P2 prolongation and correction onto the finest level as one block per
// smoother work item: the coarse planes the item needs (its 16 x 4 coarse
// footprint with a 1-cell halo, planes z0/2 - 1 .. z1/2) are staged in LDS
// once; thread (u, v) owns one fine column, issues the loads of its whole
// column first, then adds the interpolated correction on active cells (same
// weights and summation order as prolong_col).  Fine loads and stores are
// masked by the item's activity masks.
template <typename T, int SEGZ>
__global__ __launch_bounds__(NT) void k_prolong_march(const uint8_t *__restrict__ code, const T *__restrict__ xc,
                                                      int cnx, int cny, int cnz, T *__restrict__ x, int nx, int ny,
                                                      int nz, const Seg *__restrict__ segs,
                                                      const unsigned long long *__restrict__ pm, int nsegs,
                                                      const int *__restrict__ halt) {
    constexpr int CX = TX / 2 + 2, CY = TY / 2 + 2, CP = CX * CY;
    constexpr int NCZ = SEGZ / 2 + 2;
    __shared__ T cs[NCZ][CP];
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= nsegs || (halt && *halt)) return;
    const Seg sg = segs[item];
    const int tid = threadIdx.x;
    const unsigned long long *im = pm + (size_t)item * (SEGZ + 4);
    const int z0 = max(sg.z0, 0), z1 = min(sg.z1, nz);  // even (tile-aligned, even dims)
    const int I0 = sg.x0 / 2 - 1, J0 = sg.y0 / 2 - 1, K0 = z0 / 2 - 1;
    const size_t cpl = (size_t)cnx * cny, pl = (size_t)nx * ny;
    for (int e = tid; e < NCZ * CP; e += NT) {
        const int kz = e / CP, r = e - kz * CP;
        const int ci = I0 + r % CX, cj = J0 + r / CX, K = K0 + kz;
        const bool ok = ci >= 0 && ci < cnx && cj >= 0 && cj < cny && K >= 0 && K < cnz;
        const size_t P = (size_t)clampi(K, cnz - 1) * cpl + (size_t)clampi(cj, cny - 1) * cnx + clampi(ci, cnx - 1);
        const T vv = xc[P];
        cs[kz][r] = ok ? vv : T(0);
    }
    const int u = tid % TX, v = tid / TX;
    const int i = sg.x0 + u, j = sg.y0 + v;
    const bool own = i < nx && j < ny;
    const int c0 = own ? j * nx + i : 0;
    const int mb = item_mask_bit(u + 2, v + 2);
    const int pbytes = (int)(pl * sizeof(T));
    T xv[SEGZ];
    uint8_t cv[SEGZ];
    int oq[SEGZ];  // own cell's element offset per plane, OFF_NONE when masked
#pragma unroll
    for (int q = 0; q < SEGZ; q++) {
        const int k = z0 + q;
        const bool ld = own && k < z1 && ((im[q + 2] >> mb) & 1ull);
        oq[q] = ld ? c0 : OFF_NONE;
        const size_t b = (size_t)min(k, nz - 1) * pl;
        xv[q] = bload<T>(rsrc(x + b, pbytes), ld ? c0 * (int)sizeof(T) : OFF_NONE);
        cv[q] = bload<uint8_t>(rsrc(code + b, (int)pl), oq[q]);
    }
    __syncthreads();
    const int a0 = u / 2 + 1, b0 = v / 2 + 1;  // parent in the staged footprint
    const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1;
    const T w4[2] = {T(0.75), T(0.25)};
#pragma unroll
    for (int q = 0; q < SEGZ; q++) {
        const int k = z0 + q;
        if (!own || k >= z1 || cv[q] == CODE_OFF) continue;
        const int pk = (k >> 1) - K0;
        const int nk = pk + ((k & 1) ? 1 : -1);
        T s = T(0);
#pragma unroll
        for (int cz = 0; cz < 2; cz++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int a = 0; a < 2; a++)
                    s += w4[a] * w4[b] * w4[cz] * cs[cz ? nk : pk][(b0 + b * sy) * CX + (a0 + a * sx)];
        bstore<T>(xv[q] + s, rsrc(x + (size_t)k * pl, pbytes), oq[q] * (int)sizeof(T));
    }
}

template <typename T, bool FINE>
__global__ __launch_bounds__(NT) void k_prolong(const int *__restrict__ tiles, int ntiles, int ntx, int nty, int nx,
                                                int ny, int nz, const uint8_t *__restrict__ code,
                                                const T *__restrict__ dco, const T *__restrict__ xc, int cnx, int cny,
                                                int cnz, T *__restrict__ x, const int *__restrict__ halt) {
    int tile, q, w;
    if (!block_tile(tiles, ntiles, NQ, tile, q, w, halt)) return;
    prolong_col<T, FINE>(tile_col(tile, q, ntx, nty, nx, ny), nx, ny, nz, code, dco, xc, cnx, cny, cnz, x);
}

template <typename T>
__global__ __launch_bounds__(NT) void k_zero_tiles(const int *__restrict__ tiles, int ntiles, int ntx, int nty, int nx,
                                                   int ny, int nz, T *__restrict__ x, const int *__restrict__ halt) {
    int tile, kk, w;
    if (!block_tile(tiles, ntiles, TZ, tile, kk, w, halt)) return;
    const TileCoord t = tile_cell(tile, kk, ntx, nty, nx, ny, nz);
    if (t.ok) x[(size_t)t.k * nx * ny + (size_t)t.j * nx + t.i] = T(0);
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

// The halt flag is written only by a k_finalize that runs the stop test; the
// other kernels of a cycle read it (a const view of the same flag).
inline int *halt_rw(const Level &L) { return const_cast<int *>(L.halt); }

void launch_resnorm(const Level &L, int level, const OrderData &od, const double *x, const double *f, double *part,
                    double *out, int slot, hipStream_t s, const StopTest *stop, double *host_out) {
    const double ih2 = 1.0 / (L.h * L.h);
    if (level == 0) {
        if (od.nsegs)
            with_fine_depth(od.depth, [&](auto Z) {
                k_residual_march<double, decltype(Z)::value, RM_NORM><<<grid8(od.nsegs), NT, 0, s>>>(
                    x, f, L.code, L.nx, L.ny, L.nz, ih2, od.segs, od.pmask, od.nsegs, nullptr, 0, 0, nullptr, part,
                    nullptr, nullptr, nullptr, L.halt);
            });
        k_finalize<<<1, 1024, 0, s>>>(part, od.nsegs, out, slot, const_cast<StopTest *>(stop), halt_rw(L), host_out);
        return;
    }
    if (od.ntiles)
        k_resnorm<false, true, false><<<gridc(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny,
                                                                      L.nz, ih2, nullptr, od.d, x, f, part, nullptr);
    k_finalize<<<1, 1024, 0, s>>>(part, od.ntiles * NQ, out, slot, const_cast<StopTest *>(stop), halt_rw(L),
                                  host_out);
}

void launch_finalize(const Level &L, const double *part, int n, double *out, int slot, const StopTest *stop,
                     hipStream_t s, double *host_out) {
    k_finalize<<<1, 1024, 0, s>>>(part, n, out, slot, const_cast<StopTest *>(stop), halt_rw(L), host_out);
}

void launch_set_halt(int *halt, int v, hipStream_t s) { k_set_halt<<<1, 1, 0, s>>>(halt, v); }

void launch_set_stop(StopTest *st, double thresh, double rprev, double eta, int check_switch, hipStream_t s) {
    k_set_stop<<<1, 1, 0, s>>>(st, thresh, rprev, eta, check_switch);
}

void launch_resnorm32(const Level &L, const OrderData &od, const double *x, const double *f, float *r32, double *part,
                      double *out, int slot, hipStream_t s) {
    const double ih2 = 1.0 / (L.h * L.h);
    if (od.nsegs)
        with_fine_depth(od.depth, [&](auto Z) {
            k_residual_march<double, decltype(Z)::value, RM_NORM32><<<grid8(od.nsegs), NT, 0, s>>>(
                x, f, L.code, L.nx, L.ny, L.nz, ih2, od.segs, od.pmask, od.nsegs, nullptr, 0, 0, nullptr, part, r32,
                nullptr, nullptr, L.halt);
        });
    k_finalize<<<1, 1024, 0, s>>>(part, od.nsegs, out, slot, nullptr, halt_rw(L));
}

void launch_axpy_resnorm32(const Level &L, const OrderData &od, const double *x, const float *e, double *xo,
                           const double *f, float *r32, double *part, double *out, int slot, hipStream_t s,
                           const StopTest *stop, double *host_out) {
    const double ih2 = 1.0 / (L.h * L.h);
    if (od.nsegs)
        with_fine_depth(od.depth, [&](auto Z) {
            k_residual_march<double, decltype(Z)::value, RM_AXPY32><<<grid8(od.nsegs), NT, 0, s>>>(
                x, f, L.code, L.nx, L.ny, L.nz, ih2, od.segs, od.pmask, od.nsegs, nullptr, 0, 0, nullptr, part, r32, e,
                xo, L.halt);
        });
    k_finalize<<<1, 1024, 0, s>>>(part, od.nsegs, out, slot, const_cast<StopTest *>(stop), halt_rw(L), host_out);
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
    if (level == 0) {
        const OrderData &fo = L.od[2];
        if (fo.nsegs)
            with_fine_depth(fo.depth, [&](auto Z) {
                k_residual_march<double, decltype(Z)::value, RM_RESTRICT><<<grid8(fo.nsegs), NT, 0, s>>>(
                    x, f, L.code, L.nx, L.ny, L.nz, ih2, fo.segs, fo.pmask, fo.nsegs, co.d, C.nx, C.ny, fc, nullptr,
                    nullptr, nullptr, nullptr, L.halt);
            });
    } else
        k_restrict<double, false><<<gridt(co.ntiles), NT, 0, s>>>(co.tiles, co.ntiles, C.ntx, C.nty, C.nx, C.ny,
                                                                  C.nz, co.d, L.nx, L.ny, L.nz, ih2, nullptr,
                                                                  L.od[order].d, x, f, fc, L.halt);
}

void launch_restrict32(const Level &L, const Level &C, int level, int order, const float *x, const float *f,
                       float *fc, hipStream_t s) {
    const OrderData &co = C.od[order];
    if (!co.ntiles) return;
    const float ih2 = (float)(1.0 / (L.h * L.h));
    if (level == 0) {
        const OrderData &fo = L.od[2];
        if (fo.nsegs)
            with_fine_depth(fo.depth, [&](auto Z) {
                k_residual_march<float, decltype(Z)::value, RM_RESTRICT><<<grid8(fo.nsegs), NT, 0, s>>>(
                    x, f, L.code, L.nx, L.ny, L.nz, ih2, fo.segs, fo.pmask, fo.nsegs, co.d32, C.nx, C.ny, fc, nullptr,
                    nullptr, nullptr, nullptr, L.halt);
            });
    } else
        k_restrict<float, false><<<gridt(co.ntiles), NT, 0, s>>>(co.tiles, co.ntiles, C.ntx, C.nty, C.nx, C.ny, C.nz,
                                                                 co.d32, L.nx, L.ny, L.nz, ih2, nullptr,
                                                                 L.od[order].d32, x, f, fc, L.halt);
}

void launch_prolong(const Level &L, const Level &C, int level, int order, const double *xc, double *x,
                    hipStream_t s) {
    const OrderData &od = L.od[level == 0 ? 2 : order];
    if (!od.ntiles) return;
    if (level == 0) {
        if (od.nsegs)
            with_fine_depth(od.depth, [&](auto Z) {
                k_prolong_march<double, decltype(Z)::value><<<grid8(od.nsegs), NT, 0, s>>>(
                    L.code, xc, C.nx, C.ny, C.nz, x, L.nx, L.ny, L.nz, od.segs, od.pmask, od.nsegs, L.halt);
            });
    } else
        k_prolong<double, false><<<gridc(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz,
                                                                 nullptr, od.d, xc, C.nx, C.ny, C.nz, x, L.halt);
}

void launch_prolong32(const Level &L, const Level &C, int level, int order, const float *xc, float *x,
                      hipStream_t s) {
    const OrderData &od = L.od[level == 0 ? 2 : order];
    if (!od.ntiles) return;
    if (level == 0) {
        if (od.nsegs)
            with_fine_depth(od.depth, [&](auto Z) {
                k_prolong_march<float, decltype(Z)::value><<<grid8(od.nsegs), NT, 0, s>>>(
                    L.code, xc, C.nx, C.ny, C.nz, x, L.nx, L.ny, L.nz, od.segs, od.pmask, od.nsegs, L.halt);
            });
    } else
        k_prolong<float, false><<<gridc(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz,
                                                                nullptr, od.d32, xc, C.nx, C.ny, C.nz, x, L.halt);
}

void launch_zero_tiles(const Level &L, const OrderData &od, double *x, hipStream_t s) {
    if (!od.ntiles) return;
    k_zero_tiles<double><<<gridt(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz, x,
                                                         L.halt);
}

void launch_zero_tiles32(const Level &L, const OrderData &od, float *x, hipStream_t s) {
    if (!od.ntiles) return;
    k_zero_tiles<float><<<gridt(od.ntiles), NT, 0, s>>>(od.tiles, od.ntiles, L.ntx, L.nty, L.nx, L.ny, L.nz, x,
                                                        L.halt);
}

}  // namespace mg
