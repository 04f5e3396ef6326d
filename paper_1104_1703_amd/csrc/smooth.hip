// Masked red-black Gauss-Seidel smoother (Sec. 2: red-black ordering of the
// 7-point Laplacian; Sec. 3: ghost-modified operator near the boundary).
//
// One launch performs one full pass (red half-sweep, then black) over the
// active segments of a level.  Relaxing an active cell i solves its own
// equation (1/h^2)(sum_{j active} x_j - d_i x_i) = f_i for x_i; inactive
// cells hold x = 0, so the neighbour sum runs over all six neighbours.
//
// Work item: a TX x TY column of cells marching up a z range.  The block keeps
// a ring of four planes in LDS: x with a 2-cell xy halo, f and the diagonal
// (or the finest-level neighbour code) with a 1-cell halo.  At step k it
// relaxes red cells of plane k+1 on the tile plus a 1-cell ring (redundantly
// with the neighbouring work items, from identical inputs), then black cells
// of plane k on the tile, and writes plane k.  Red cells only read black ones
// and vice versa, so each plane is updated in place; reads come from `xin`
// and writes go to `xout` (ping-pong), so concurrent work items never see
// each other's results.  Global loads of the planes needed two and three
// steps ahead are in flight in registers while a step computes, so the
// compute phases touch LDS only.  Loads go through buffer resources and are
// masked per 16-cell row granule by the item's precomputed activity masks:
// granules without an active cell (outside the domain, inside holes, halo rows
// of inactive neighbours) are never fetched, and inactive cells are never
// stored.  Net HBM traffic per pass: one read of x, f and the code/diagonal
// and one write of x, on granules holding active cells.
#include <hip/hip_ext.h>

#include "cube_core.h"
#include "mg_core.h"
#include "smooth2_core.h"
#include "smooth_res_core.h"
#include "transfer_core.h"

namespace mg {

namespace {

using namespace rb;

// Five blocks per CU (LDS); the finest float passes (16-19 KB of LDS, 62
// registers) eight, so that the 2048 items of a 256^3 pass run in one round.
template <typename T, bool FINE, int SEGZ, bool PRO = false>
__global__ __launch_bounds__(NT, FINE && sizeof(T) == 4 ? 8 : 5) void k_rbgs(
    const T *__restrict__ xin, T *__restrict__ xout, const T *__restrict__ f, const uint8_t *__restrict__ code,
    const T *__restrict__ dco, int nx, int ny, int nz, T h2, const Seg *__restrict__ segs,
    const unsigned long long *__restrict__ pm, int nsegs, const int *__restrict__ halt, const T *__restrict__ xc = nullptr,
    int cnx = 0, int cny = 0, int cnz = 0) {
    __shared__ RbgsLds<T, FINE, PRO> lds;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= nsegs || (halt && *halt)) return;
    rbgs_item<T, FINE, SEGZ, PRO>(lds, xin, xout, f, code, dco, nx, ny, nz, h2, segs[item],
                                  pm + (size_t)item * (SEGZ + 4), xc, cnx, cny, cnz);
}

// The finest pass that also forms the residual-norm partials of its input,
// one per work item, as the residual-norm march does.
template <int SZ>
__global__ __launch_bounds__(NT, 5) void k_rbgs_norm(const double *__restrict__ xin, double *__restrict__ xout,
                                                   const double *__restrict__ f, const uint8_t *__restrict__ code,
                                                   int nx, int ny, int nz, double h2, double ih2,
                                                   const Seg *__restrict__ segs,
                                                   const unsigned long long *__restrict__ pm, int nsegs,
                                                   const int *__restrict__ halt, double *__restrict__ part) {
    __shared__ RbgsLds<double, true, false> lds;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= nsegs || (halt && *halt)) return;
    const double sq = rbgs_item<double, true, SZ, false, true>(lds, xin, xout, f, code, nullptr, nx, ny, nz, h2,
                                                               segs[item], pm + (size_t)item * (SZ + 4), nullptr, 0,
                                                               0, 0, ih2);
    const double t = tr::block_sum(sq);
    if (threadIdx.x == 0) part[item] = t;
}

// The finest pass that also forms the residual of its result and restricts
// it onto level 1 (smooth_res_core.h): four FP64 blocks per CU (LDS), six
// FP32 blocks.
template <typename T, int SEGZ>
__global__ __launch_bounds__(NT, sizeof(T) == 8 ? 4 : 6) void k_rbgs_res(
    const T *__restrict__ xin, T *__restrict__ xout, const T *__restrict__ f, const uint8_t *__restrict__ code, int nx,
    int ny, int nz, T h2, T ih2, const Seg *__restrict__ segs, const unsigned long long *__restrict__ pm, int nsegs,
    const int *__restrict__ halt, const T *__restrict__ cd, int cnx, int cny, T *__restrict__ fc) {
    __shared__ rbr::Lds<T> lds;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= nsegs || (halt && *halt)) return;
    rbr::rbgs_res_item<T, SEGZ>(lds, xin, xout, f, code, nx, ny, nz, h2, ih2, segs[item],
                                          pm + (size_t)item * (SEGZ + 2 * rbr::H), cd, cnx, cny, fc);
}

// Two passes per launch (smooth2_core.h): LDS allows two FP64 blocks per CU.
template <typename T, bool FINE, int SEGZ, bool PRO = false>
__global__ __launch_bounds__(NT, 2) void k_rbgs2(const T *__restrict__ xin, T *__restrict__ xout,
                                               const T *__restrict__ f, const uint8_t *__restrict__ code,
                                               const T *__restrict__ dco, int nx, int ny, int nz, T h2,
                                               const Seg *__restrict__ segs, const unsigned long long *__restrict__ pm,
                                               int nsegs, const int *__restrict__ halt,
                                               const T *__restrict__ xc = nullptr, int cnx = 0, int cny = 0,
                                               int cnz = 0) {
    __shared__ rb2::Lds<T, FINE, PRO> lds;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= nsegs || (halt && *halt)) return;
    rb2::rbgs2_item<T, FINE, SEGZ, PRO>(lds, xin, xout, f, code, dco, nx, ny, nz, h2, segs[item],
                                        pm + (size_t)item * (SEGZ + 2 * rb2::H), xc, cnx, cny, cnz);
}

// Coarse-level pass over 8 x 8 x 8 cubes (four per active 32 x 8 x 8 tile),
// each loaded whole: cube_core.h.
template <typename T>
__global__ __launch_bounds__(cube::NT) void k_rbgs_cube(const T *__restrict__ xin, T *__restrict__ xout,
                                                      const T *__restrict__ f, const T *__restrict__ d, int nx, int ny,
                                                      int nz, int ntx, int nty, T h2, const int *__restrict__ tiles,
                                                      int ntiles, const int *__restrict__ halt) {
    __shared__ cube::Lds<T> lds;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= 4 * ntiles || (halt && *halt)) return;
    const int tile = tiles[item >> 2];
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    const int x0 = tx * TX + (item & 3) * cube::C;
    if (x0 >= nx) return;  // a tile wider than the level
    cube::rbgs_cube<T>(lds, xin, xout, f, d, nx, ny, nz, h2, x0, ty * TY, tz * TZ);
}

// The cube pass that also forms the residual and its R1 restriction onto
// the next coarser level (the last pre-smoothing pass of a cube level).
template <typename T>
__global__ __launch_bounds__(cube::NT) void k_rbgs_cube_restrict(
    const T *__restrict__ xin, T *__restrict__ xout, const T *__restrict__ f, const T *__restrict__ d, int nx, int ny,
    int nz, int ntx, int nty, T h2, T ih2, const int *__restrict__ tiles, int ntiles, const int *__restrict__ halt,
    const T *__restrict__ cd, T *__restrict__ fc, int cnx, int cny, int cnz) {
    __shared__ cube::LdsRes<T> lds;
    const int item = xcd_item(blockIdx.x, gridDim.x);
    if (item >= 4 * ntiles || (halt && *halt)) return;
    const int tile = tiles[item >> 2];
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
    const int x0 = tx * TX + (item & 3) * cube::C;
    if (x0 >= nx) return;  // a tile wider than the level
    cube::rbgs_cube_restrict<T>(lds, xin, xout, f, d, nx, ny, nz, h2, ih2, x0, ty * TY, tz * TZ, cd, fc, cnx, cny,
                                cnz);
}

inline unsigned grid8(int items) { return (unsigned)(((items + 7) / 8) * 8); }

template <typename T>
struct same_t {
    using type = T;
};
// Launches kernel k over `grid` blocks of NT threads; with events, through
// hipExtLaunchKernel so that e0 and e1 take the kernel's own start and end.
template <typename... P>
hipError_t launch_k(void (*k)(P...), unsigned grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                    typename same_t<P>::type... a) {
    if (!e0 && !e1) {
        k<<<grid, NT, 0, s>>>(a...);
        return hipSuccess;
    }
    void *args[] = {(void *)&a...};
    return hipExtLaunchKernel((const void *)k, dim3(grid), dim3(NT), args, 0, s, e0, e1, 0);
}

}  // namespace

template <typename T>
void launch_cube_restrict(const T *xin, T *xout, const T *f, const T *d, const Level &L, const OrderData &od, T h2,
                          T ih2, const Level &C, const T *cd, T *fc, hipStream_t s) {
    if (od.ntiles == 0) return;
    k_rbgs_cube_restrict<T><<<grid8(4 * od.ntiles), cube::NT, 0, s>>>(xin, xout, f, d, L.nx, L.ny, L.nz, L.ntx,
                                                                     L.nty, h2, ih2, od.tiles, od.ntiles, L.halt, cd,
                                                                     fc, C.nx, C.ny, C.nz);
}

void launch_rbgs_restrict(const Level &L, const Level &C, int order, const OrderData &od, const double *xin,
                          double *xout, const double *f, double *fc, hipStream_t s) {
    launch_cube_restrict<double>(xin, xout, f, od.d, L, od, L.h * L.h, 1.0 / (L.h * L.h), C, C.od[order].d, fc, s);
}

void launch_rbgs_restrict32(const Level &L, const Level &C, int order, const OrderData &od, const float *xin,
                            float *xout, const float *f, float *fc, hipStream_t s) {
    launch_cube_restrict<float>(xin, xout, f, od.d32, L, od, (float)(L.h * L.h), (float)(1.0 / (L.h * L.h)), C,
                                C.od[order].d32, fc, s);
}

template <typename T>
hipError_t launch_fine_res(const Level &L, const OrderData &od, const T *xin, T *xout, const T *f, const Level &C,
                           const T *cd, T *fc, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (od.nsegs == 0) return hipSuccess;
    const T h2 = (T)(L.h * L.h), ih2 = (T)(1.0 / (L.h * L.h));
    hipError_t err = hipSuccess;
    with_fine_depth(od.depth, [&](auto Z) {
        err = launch_k(k_rbgs_res<T, decltype(Z)::value>, grid8(od.nsegs), s, e0, e1, xin, xout, f, L.code, L.nx,
                       L.ny, L.nz, h2, ih2, od.segs, od.pmask3, od.nsegs, L.halt, cd, C.nx, C.ny, fc);
    });
    return err;
}

hipError_t launch_rbgs_res_fine(const Level &L, const Level &C, int order, const OrderData &od, const double *xin,
                                double *xout, const double *f, double *fc, hipStream_t s, hipEvent_t e0,
                                hipEvent_t e1) {
    return launch_fine_res<double>(L, od, xin, xout, f, C, C.od[order].d, fc, s, e0, e1);
}

hipError_t launch_rbgs_res_fine32(const Level &L, const Level &C, int order, const OrderData &od, const float *xin,
                                  float *xout, const float *f, float *fc, hipStream_t s, hipEvent_t e0,
                                  hipEvent_t e1) {
    return launch_fine_res<float>(L, od, xin, xout, f, C, C.od[order].d32, fc, s, e0, e1);
}

template <typename T>
void launch_cube(const T *xin, T *xout, const T *f, const T *d, const Level &L, const OrderData &od, T h2,
                 hipStream_t s) {
    static_assert(TX == 4 * cube::C && TY == cube::C && TZ == cube::C, "a tile holds four cubes");
    if (od.ntiles == 0) return;
    k_rbgs_cube<T><<<grid8(4 * od.ntiles), cube::NT, 0, s>>>(xin, xout, f, d, L.nx, L.ny, L.nz, L.ntx, L.nty, h2,
                                                            od.tiles, od.ntiles, L.halt);
}

// Coarse levels: the kernel instance for the level's item depth.
template <typename T, bool PRO = false>
void launch_coarse(int depth, const T *xin, T *xout, const T *f, const T *d, const Level &L, const OrderData &od,
                   T h2, hipStream_t s, const T *xc = nullptr, const Level *C = nullptr) {
    const int cnx = C ? C->nx : 0, cny = C ? C->ny : 0, cnz = C ? C->nz : 0;
    if (depth == 8)
        k_rbgs<T, false, 8, PRO><<<grid8(od.nsegs), NT, 0, s>>>(xin, xout, f, nullptr, d, L.nx, L.ny, L.nz, h2,
                                                               od.segs, od.pmask, od.nsegs, L.halt, xc, cnx, cny, cnz);
    else if (depth == 2)
        k_rbgs<T, false, 2, PRO><<<grid8(od.nsegs), NT, 0, s>>>(xin, xout, f, nullptr, d, L.nx, L.ny, L.nz, h2,
                                                               od.segs, od.pmask, od.nsegs, L.halt, xc, cnx, cny, cnz);
    else
        k_rbgs<T, false, 4, PRO><<<grid8(od.nsegs), NT, 0, s>>>(xin, xout, f, nullptr, d, L.nx, L.ny, L.nz, h2,
                                                               od.segs, od.pmask, od.nsegs, L.halt, xc, cnx, cny, cnz);
}
static_assert((SEGZ_COARSE1 == 2 || SEGZ_COARSE1 == 4 || SEGZ_COARSE1 == 8) &&
                  (SEGZ_COARSE == 2 || SEGZ_COARSE == 4 || SEGZ_COARSE == 8),
              "coarse item depths have kernel instances for 2, 4 and 8 planes");

// A finest-level pass; with events, launched so that e0 and e1 take the
// kernel's own start and end times.
template <typename T>
hipError_t launch_fine(const Level &L, const OrderData &od, const T *xin, T *xout, const T *f, T h2, hipStream_t s,
                       hipEvent_t e0, hipEvent_t e1) {
    hipError_t err = hipSuccess;
    with_fine_depth(od.depth, [&](auto Z) {
        err = launch_k(k_rbgs<T, true, decltype(Z)::value>, grid8(od.nsegs), s, e0, e1, xin, xout, f, L.code,
                       (const T *)nullptr, L.nx, L.ny, L.nz, h2, od.segs, od.pmask, od.nsegs, L.halt,
                       (const T *)nullptr, 0, 0, 0);
    });
    return err;
}

hipError_t launch_rbgs(const Level &L, int level, const OrderData &od, const double *xin, double *xout,
                       const double *f, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (od.nsegs == 0) return hipSuccess;
    const double h2 = L.h * L.h;
    if (level == 0)
        return launch_fine<double>(L, od, xin, xout, f, h2, s, e0, e1);
    else if (od.cube)
        launch_cube<double>(xin, xout, f, od.d, L, od, h2, s);
    else
        launch_coarse<double>(od.depth, xin, xout, f, od.d, L, od, h2, s);
    return hipSuccess;
}

hipError_t launch_rbgs_norm(const Level &L, const OrderData &od, const double *xin, double *xout, const double *f,
                            double *part, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (od.nsegs == 0) return hipSuccess;
    hipError_t err = hipSuccess;
    with_fine_depth(od.depth, [&](auto Z) {
        err = launch_k(k_rbgs_norm<decltype(Z)::value>, grid8(od.nsegs), s, e0, e1, xin, xout, f, L.code, L.nx, L.ny,
                       L.nz, L.h * L.h, 1.0 / (L.h * L.h), od.segs, od.pmask, od.nsegs, L.halt, part);
    });
    return err;
}

hipError_t launch_rbgs_prolong(const Level &L, int level, const OrderData &od, const Level &C, const double *xc,
                               const double *xin, double *xout, const double *f, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1) {
    if (od.nsegs == 0) return hipSuccess;
    const double h2 = L.h * L.h;
    hipError_t err = hipSuccess;
    if (level == 0)
        with_fine_depth(od.depth, [&](auto Z) {
            err = launch_k(k_rbgs<double, true, decltype(Z)::value, true>, grid8(od.nsegs), s, e0, e1, xin, xout, f,
                           L.code, (const double *)nullptr, L.nx, L.ny, L.nz, h2, od.segs, od.pmask, od.nsegs, L.halt,
                           xc, C.nx, C.ny, C.nz);
        });
    else if (level == 1 && od.nsegs8 > 0)  // whole tiles: one round at 4 blocks per CU
        k_rbgs<double, false, TZ, true><<<grid8(od.nsegs8), NT, 0, s>>>(xin, xout, f, nullptr, od.d, L.nx, L.ny, L.nz,
                                                                      h2, od.segs8, od.pmask8, od.nsegs8, L.halt, xc,
                                                                      C.nx, C.ny, C.nz);
    else
        launch_coarse<double, true>(od.depth, xin, xout, f, od.d, L, od, h2, s, xc, &C);
    return err;
}

hipError_t launch_rbgs_prolong32(const Level &L, int level, const OrderData &od, const Level &C, const float *xc,
                                 const float *xin, float *xout, const float *f, hipStream_t s, hipEvent_t e0,
                                 hipEvent_t e1) {
    if (od.nsegs == 0) return hipSuccess;
    const float h2 = (float)(L.h * L.h);
    hipError_t err = hipSuccess;
    if (level == 0)
        with_fine_depth(od.depth, [&](auto Z) {
            err = launch_k(k_rbgs<float, true, decltype(Z)::value, true>, grid8(od.nsegs), s, e0, e1, xin, xout, f,
                           L.code, (const float *)nullptr, L.nx, L.ny, L.nz, h2, od.segs, od.pmask, od.nsegs, L.halt,
                           xc, C.nx, C.ny, C.nz);
        });
    else
        launch_coarse<float, true>(od.depth, xin, xout, f, od.d32, L, od, h2, s, xc, &C);
    return err;
}

template <typename T>
void launch_fused(const Level &L, int level, const OrderData &od, const T *xin, T *xout, const T *f, const T *d,
                  T h2, hipStream_t s) {
    if (od.nsegs == 0) return;
    const unsigned g = grid8(od.nsegs);
    if (level == 0)
        k_rbgs2<T, true, SEG_TILES_FINE * TZ><<<g, NT, 0, s>>>(xin, xout, f, L.code, nullptr, L.nx, L.ny, L.nz, h2,
                                                               od.segs, od.pmask2, od.nsegs, L.halt);
    else if (od.depth == 8)
        k_rbgs2<T, false, 8><<<g, NT, 0, s>>>(xin, xout, f, nullptr, d, L.nx, L.ny, L.nz, h2, od.segs, od.pmask2,
                                              od.nsegs, L.halt);
    else if (od.depth == 4)
        k_rbgs2<T, false, 4><<<g, NT, 0, s>>>(xin, xout, f, nullptr, d, L.nx, L.ny, L.nz, h2, od.segs, od.pmask2,
                                              od.nsegs, L.halt);
    else
        k_rbgs2<T, false, 2><<<g, NT, 0, s>>>(xin, xout, f, nullptr, d, L.nx, L.ny, L.nz, h2, od.segs, od.pmask2,
                                              od.nsegs, L.halt);
}

void launch_rbgs2(const Level &L, int level, const OrderData &od, const double *xin, double *xout, const double *f,
                  hipStream_t s) {
    launch_fused<double>(L, level, od, xin, xout, f, od.d, L.h * L.h, s);
}

void launch_rbgs2_32(const Level &L, int level, const OrderData &od, const float *xin, float *xout, const float *f,
                     hipStream_t s) {
    launch_fused<float>(L, level, od, xin, xout, f, od.d32, (float)(L.h * L.h), s);
}

void launch_rbgs2_prolong(const Level &L, const OrderData &od, const Level &C, const double *xc, const double *xin,
                          double *xout, const double *f, hipStream_t s) {
    if (od.nsegs == 0) return;
    k_rbgs2<double, true, SEG_TILES_FINE * TZ, true><<<grid8(od.nsegs), NT, 0, s>>>(
        xin, xout, f, L.code, nullptr, L.nx, L.ny, L.nz, L.h * L.h, od.segs, od.pmask2, od.nsegs, L.halt, xc, C.nx,
        C.ny, C.nz);
}

void launch_rbgs2_prolong32(const Level &L, const OrderData &od, const Level &C, const float *xc, const float *xin,
                            float *xout, const float *f, hipStream_t s) {
    if (od.nsegs == 0) return;
    k_rbgs2<float, true, SEG_TILES_FINE * TZ, true><<<grid8(od.nsegs), NT, 0, s>>>(
        xin, xout, f, L.code, nullptr, L.nx, L.ny, L.nz, (float)(L.h * L.h), od.segs, od.pmask2, od.nsegs, L.halt,
        xc, C.nx, C.ny, C.nz);
}

hipError_t launch_rbgs32(const Level &L, int level, const OrderData &od, const float *xin, float *xout,
                         const float *f, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (od.nsegs == 0) return hipSuccess;
    const float h2 = (float)(L.h * L.h);
    if (level == 0)
        return launch_fine<float>(L, od, xin, xout, f, h2, s, e0, e1);
    else if (od.cube)
        launch_cube<float>(xin, xout, f, od.d32, L, od, h2, s);
    else
        launch_coarse<float>(od.depth, xin, xout, f, od.d32, L, od, h2, s);
    return hipSuccess;
}

}  // namespace mg
