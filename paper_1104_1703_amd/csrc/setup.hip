// Hierarchy construction kernels (run once per mask).
//
// Sec. 3: the mask is +1 inside, -1 outside, and coarse masks are the R1
// average of their children.  Averages are kept as exact integer counts c of
// active finest descendants (m = 2c/8^l - 1), so the domain test m > 0 is
// 2c > 8^l and the first-order test m = 1 (Sec. 4) is c = 8^l, both exact.
#include "mg_core.h"
#include "smooth_core.h"

namespace mg {

namespace {

__global__ void k_validate(const int8_t *__restrict__ mask, int nx, int ny, int nz,
                           unsigned long long *__restrict__ bad) {
    size_t n = (size_t)nx * ny * nz;
    unsigned bad_val = 0, bad_frame = 0, act = 0;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        int v = mask[p];
        int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / ((size_t)nx * ny));
        bool frame = (i == 0 || j == 0 || k == 0 || i == nx - 1 || j == ny - 1 || k == nz - 1);
        bad_val += (v != 1 && v != -1);
        bad_frame += (frame && v != -1);
        act += (v == 1);
    }
    if (bad_val) atomicAdd(&bad[0], (unsigned long long)bad_val);
    if (bad_frame) atomicAdd(&bad[1], (unsigned long long)bad_frame);
    if (act) atomicAdd(&bad[2], (unsigned long long)act);
}

__global__ void k_count0(const int8_t *__restrict__ mask, int32_t *__restrict__ cnt, size_t n) {
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x)
        cnt[p] = (mask[p] == 1) ? 1 : 0;
}

// R1 sum of the mask counts: coarse cell I gets the sum over its 8 children.
__global__ void k_count_up(const int32_t *__restrict__ fine, int fnx, int fny, int32_t *__restrict__ coarse, int cnx,
                           int cny, int cnz) {
    size_t n = (size_t)cnx * cny * cnz;
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x) {
        int i = (int)(p % cnx), j = (int)((p / cnx) % cny), k = (int)(p / ((size_t)cnx * cny));
        int32_t s = 0;
#pragma unroll
        for (int c = 0; c < 8; c++) {
            int a = 2 * i + (c & 1), b = 2 * j + ((c >> 1) & 1), e = 2 * k + (c >> 2);
            s += fine[((size_t)e * fny + b) * fnx + a];
        }
        coarse[p] = s;
    }
}

__device__ __forceinline__ bool is_active(int32_t c, int level, int order) {
    if (level == 0) return c == 1;
    const int64_t N = (int64_t)1 << (3 * level);
    return order == 2 ? (2 * (int64_t)c > N) : ((int64_t)c == N);
}

// Finest level: with the boundary on the face (theta = 1/2) the diagonal of an
// active cell's equation is (#active) + 2 (#inactive) = 12 - (#active face
// neighbours); the code holds it (6..12), CODE_OFF (0) for an inactive cell,
// so that a zero-filled (skipped) load reads as inactive.
__global__ void k_code0(const int32_t *__restrict__ cnt, int nx, int ny, int nz, uint8_t *__restrict__ code,
                        unsigned long long *__restrict__ nact) {
    size_t n = (size_t)nx * ny * nz;
    size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    int a = 0;
    if (p < n) {
        int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / ((size_t)nx * ny));
        if (cnt[p] == 1) {
            a = 1;
            int na = 0;
            na += (i > 0 && cnt[p - 1] == 1);
            na += (i < nx - 1 && cnt[p + 1] == 1);
            na += (j > 0 && cnt[p - nx] == 1);
            na += (j < ny - 1 && cnt[p + nx] == 1);
            na += (k > 0 && cnt[p - (size_t)nx * ny] == 1);
            na += (k < nz - 1 && cnt[p + (size_t)nx * ny] == 1);
            code[p] = (uint8_t)(12 - na);
        } else {
            code[p] = CODE_OFF;
        }
    }
    int c = __syncthreads_count(a);
    if (threadIdx.x == 0 && c) atomicAdd(nact, (unsigned long long)c);
}

// Coarse diagonal (Sec. 3 ghost value; Sec. 4 first order).  For an active
// cell i and a neighbour j outside the level's domain the ghost value
// (g - (1 - theta) x_i)/theta with g = 0 puts 1/theta on the diagonal, where
// theta = m_i/(m_i - m_j) is where the linearly interpolated mask crosses 0.
// In counts: 1/theta = (2c_i - 2c_j)/(2c_i - 8^l), one correctly rounded
// division of exact integers.  First order pins every cell with m < 1 to 0
// at its centre: theta = 1.
__global__ void k_diag(const int32_t *__restrict__ cnt, int nx, int ny, int nz, int level, int order,
                       double *__restrict__ d, unsigned long long *__restrict__ nact) {
    size_t n = (size_t)nx * ny * nz;
    size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    int a = 0;
    if (p < n) {
        int i = (int)(p % nx), j = (int)((p / nx) % ny), k = (int)(p / ((size_t)nx * ny));
        const int32_t ci = cnt[p];
        double dv = 0.0;
        if (is_active(ci, level, order)) {
            a = 1;
            const int64_t N = (int64_t)1 << (3 * level);
            const size_t pl = (size_t)nx * ny;
            int32_t cj[6];
            cj[0] = i > 0 ? cnt[p - 1] : 0;
            cj[1] = i < nx - 1 ? cnt[p + 1] : 0;
            cj[2] = j > 0 ? cnt[p - nx] : 0;
            cj[3] = j < ny - 1 ? cnt[p + nx] : 0;
            cj[4] = k > 0 ? cnt[p - pl] : 0;
            cj[5] = k < nz - 1 ? cnt[p + pl] : 0;
#pragma unroll
            for (int q = 0; q < 6; q++) {
                if (is_active(cj[q], level, order)) {
                    dv += 1.0;
                } else if (order == 2) {
                    dv += (double)(2 * (int64_t)ci - 2 * (int64_t)cj[q]) / (double)(2 * (int64_t)ci - N);
                } else {
                    dv += 1.0;
                }
            }
        }
        d[p] = dv;
    }
    int c = __syncthreads_count(a);
    if (threadIdx.x == 0 && c) atomicAdd(nact, (unsigned long long)c);
}

// One block per tile: flag = 1 if any cell of the tile is active.
__global__ void k_tile_flags(const int32_t *__restrict__ cnt, int nx, int ny, int nz, int ntx, int nty, int level,
                             int order, uint8_t *__restrict__ flags) {
    int t = blockIdx.x;
    int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
    int any = 0;
    for (int e = threadIdx.x; e < TX * TY * TZ; e += blockDim.x) {
        int i = tx * TX + e % TX, j = ty * TY + (e / TX) % TY, k = tz * TZ + e / (TX * TY);
        if (i < nx && j < ny && k < nz) any |= is_active(cnt[((size_t)k * ny + j) * nx + i], level, order);
    }
    int c = __syncthreads_or(any);
    if (threadIdx.x == 0) flags[t] = (uint8_t)(c != 0);
}

// One block per smoother work item: its activity masks (one word per plane
// z0-2 .. z0+npl-3; bit layout of item_mask_bit).
// Activity masks of smoother work items with an xy halo of HH cells (2: one
// pass per launch, smooth_core.h; 3: the finest pass that also forms the
// residual, smooth_res_core.h; 4: two fused passes, smooth2_core.h): per
// item and plane z0-HH .. z0-HH+npl-1, bit 4 v + g for row y0-HH+v and the
// 16-cell granule g of the row (granule boundaries at x0-16, x0, x0+16,
// x0+32); planes outside the box or past z1+HH-1 get no bits.
template <int HH>
__global__ void k_item_masks(const int32_t *__restrict__ cnt, int nx, int ny, int nz, int level, int order,
                             const Seg *__restrict__ segs, int npl, unsigned long long *__restrict__ pm) {
    constexpr int RY = TY + 2 * HH, RX = TX + 2 * HH;
    static_assert(4 * RY <= 64, "one 64-bit word per plane");
    __shared__ unsigned rowbits[(SEGZ_FINE_MAX + 2 * HH) * RY];
    const Seg sg = segs[blockIdx.x];
    for (int r = threadIdx.x; r < npl * RY; r += blockDim.x) {
        const int pi = r / RY, v = r % RY;
        const int k = sg.z0 - HH + pi, y = sg.y0 - HH + v;
        unsigned bits = 0;
        if (k >= 0 && k < nz && k <= sg.z1 + HH - 1 && y >= 0 && y < ny)
            for (int u = 0; u < RX; u++) {
                const int x = sg.x0 - HH + u;
                if (x >= 0 && x < nx && is_active(cnt[((size_t)k * ny + y) * nx + x], level, order))
                    bits |= 1u << ((u + 16 - HH) >> 4);
            }
        rowbits[r] = bits;
    }
    __syncthreads();
    for (int pi = threadIdx.x; pi < npl; pi += blockDim.x) {
        unsigned long long w = 0;
        for (int v = 0; v < RY; v++) w |= (unsigned long long)rowbits[pi * RY + v] << (4 * v);
        pm[(size_t)blockIdx.x * npl + pi] = w;
    }
}

__global__ void k_to_float(const double *__restrict__ a, float *__restrict__ b, size_t n) {
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n; p += (size_t)gridDim.x * blockDim.x)
        b[p] = (float)a[p];
}

inline unsigned grid_for(size_t n, unsigned bs = 256) {
    size_t g = (n + bs - 1) / bs;
    if (g > 65535u * 16u) g = 65535u * 16u;
    return (unsigned)(g ? g : 1);
}

}  // namespace

void launch_validate(const int8_t *mask, int nx, int ny, int nz, unsigned long long *bad, hipStream_t s) {
    size_t n = (size_t)nx * ny * nz;
    unsigned g = grid_for(n);
    if (g > 4096) g = 4096;
    k_validate<<<g, 256, 0, s>>>(mask, nx, ny, nz, bad);
}

void launch_count0(const int8_t *mask, int32_t *cnt, size_t n, hipStream_t s) {
    k_count0<<<grid_for(n), 256, 0, s>>>(mask, cnt, n);
}

void launch_count_up(const Level &fine, const Level &coarse, hipStream_t s) {
    k_count_up<<<grid_for(coarse.n), 256, 0, s>>>(fine.cnt, fine.nx, fine.ny, coarse.cnt, coarse.nx, coarse.ny,
                                                   coarse.nz);
}

void launch_code0(const Level &L, unsigned long long *nact, hipStream_t s) {
    k_code0<<<(unsigned)((L.n + 255) / 256), 256, 0, s>>>(L.cnt, L.nx, L.ny, L.nz, L.code, nact);
}

void launch_diag(const Level &L, int level, int order, double *d, unsigned long long *nact, hipStream_t s) {
    k_diag<<<(unsigned)((L.n + 255) / 256), 256, 0, s>>>(L.cnt, L.nx, L.ny, L.nz, level, order, d, nact);
}

void launch_tile_flags(const Level &L, int level, int order, uint8_t *flags, hipStream_t s) {
    int nt = L.ntx * L.nty * L.ntz;
    k_tile_flags<<<nt, 256, 0, s>>>(L.cnt, L.nx, L.ny, L.nz, L.ntx, L.nty, level, order, flags);
}

void launch_item_masks(const Level &L, int level, int order, const OrderData &od, int npl, unsigned long long *pm,
                       hipStream_t s, int halo) {
    if (od.nsegs == 0) return;
    if (halo == 4)
        k_item_masks<4><<<od.nsegs, 256, 0, s>>>(L.cnt, L.nx, L.ny, L.nz, level, order, od.segs, npl, pm);
    else if (halo == 3)
        k_item_masks<3><<<od.nsegs, 256, 0, s>>>(L.cnt, L.nx, L.ny, L.nz, level, order, od.segs, npl, pm);
    else
        k_item_masks<2><<<od.nsegs, 256, 0, s>>>(L.cnt, L.nx, L.ny, L.nz, level, order, od.segs, npl, pm);
}

void launch_to_float(const double *a, float *b, size_t n, hipStream_t s) {
    k_to_float<<<grid_for(n), 256, 0, s>>>(a, b, n);
}

}  // namespace mg
