// Small coarse levels in one workgroup.
//
// Below a few thousand cells a level is far too small to fill the GPU, and
// one launch per half-sweep would cost more than the work.  This kernel runs
// one whole multigrid call MG(ls) (Sec. 2 enumerated recipe, with N_cycles
// recursive calls per level and n_coarse passes on the deepest level) for the
// levels ls..last inside one 1024-thread workgroup, with every level's x, f
// and diagonal resident in LDS.  Red-black Gauss-Seidel is done in place with
// a barrier between the colours (a colour only reads the other colour).
#include <algorithm>

#include "coarse_core.h"

namespace mg {

namespace {

using namespace small;

constexpr int NTC = 1024;  // 16 waves: four per SIMD to hide LDS and FP64 latency

template <typename T>
__global__ __launch_bounds__(NTC) void k_coarse(SmallLevels<T> S) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if (S.halt && *S.halt) return;
    small_tail<T, NTC>(reinterpret_cast<T *>(smem_raw), S, S.f0, S.x0, S.load_x != 0);
}

template <typename T>
void launch_impl(const mg_hierarchy *H, int order, int ls, bool zero_start, const T *f0, T *x0, hipStream_t s,
                 bool f32) {
    SmallLevels<T> S{};
    const int last = H->nlev[order] - 1;
    S.n = last - ls + 1;
    int off = 0;
    for (int q = 0; q < S.n; q++) {
        const Level &L = H->lev[ls + q];
        S.nx[q] = L.nx;
        S.ny[q] = L.ny;
        S.nz[q] = L.nz;
        S.mx[q] = div_magic((unsigned)L.nx);
        S.mxy[q] = div_magic((unsigned)(L.nx * L.ny));
        S.mh[q] = div_magic((unsigned)((L.nx + 1) / 2));
        S.mhy[q] = div_magic((unsigned)((L.nx + 1) / 2 * L.ny));
        S.h2[q] = (T)(L.h * L.h);
        S.ih2[q] = (T)(1.0 / (L.h * L.h));
        S.d[q] = f32 ? (const T *)L.od[order].d32 : (const T *)L.od[order].d;
        S.off[q] = off;
        off += 3 * (int)L.n;
    }
    S.f0 = f0;
    S.x0 = x0;
    S.load_x = zero_start ? 0 : 1;
    S.halt = H->lev[0].halt;
    S.n_pre = H->opt.n_pre;
    S.n_post = H->opt.n_post;
    S.n_cycles = H->opt.n_cycles;
    S.n_coarse = H->opt.n_coarse_sweeps;
    const size_t bytes = (size_t)off * sizeof(T);
    k_coarse<T><<<1, NTC, bytes, s>>>(S);
}

}  // namespace

size_t small_lds_bytes(const mg_hierarchy *H, int order, int ls, bool f32) {
    size_t n = 0;
    for (int l = ls; l < H->nlev[order]; l++) n += 3 * H->lev[l].n;
    return n * (f32 ? sizeof(float) : sizeof(double));
}

// Largest dynamic LDS the one-workgroup kernel may use on the current device
// (0 if it cannot run).  Any refused request is cleared so that no error is
// left pending for the caller's next HIP call.
int small_init() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    int lim = std::min(v, SMALL_LDS_MAX) - 1024;  // room for the kernel's static LDS
    if (lim > 64 * 1024 - 1024) {
        if (hipFuncSetAttribute((const void *)k_coarse<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) !=
                hipSuccess ||
            hipFuncSetAttribute((const void *)k_coarse<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lim) !=
                hipSuccess) {
            (void)hipGetLastError();
            lim = 64 * 1024 - 1024;
        }
    }
    return lim > 0 ? lim : 0;
}

void launch_small(const mg_hierarchy *H, int order, int ls, bool zero_start, const double *f0, double *x0,
                  hipStream_t s) {
    launch_impl<double>(H, order, ls, zero_start, f0, x0, s, false);
}

void launch_small32(const mg_hierarchy *H, int order, int ls, bool zero_start, const float *f0, float *x0,
                    hipStream_t s) {
    launch_impl<float>(H, order, ls, zero_start, f0, x0, s, true);
}

}  // namespace mg
