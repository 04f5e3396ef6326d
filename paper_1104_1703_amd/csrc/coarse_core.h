// Core of the one-workgroup multigrid call on small levels, shared by the
// per-level path (coarse.hip) and the batched phase kernels (batch.hip).
#pragma once

#include "mg_core.h"
#include "smooth_core.h"

namespace mg {
namespace small {

template <typename T>
struct SmallLevels {
    int n;                 // number of levels held (ls..last)
    int nx[MAXS], ny[MAXS], nz[MAXS];
    unsigned long long mx[MAXS], mxy[MAXS];  // division magics, see qdiv
    unsigned long long mh[MAXS], mhy[MAXS];  // ... of hx = ceil(nx / 2) and hx * ny
    T h2[MAXS];            // h^2 per level
    T ih2[MAXS];           // 1/h^2 per level
    const T *d[MAXS];      // diagonal per level (global), 0 off the domain
    int off[MAXS];         // LDS offset (elements) of the level's x; f and d follow
    const T *f0;           // right-hand side of level ls (global)
    T *x0;                 // iterate of level ls (global, in/out)
    int load_x;            // 1: start from x0, 0: start from zero
    const int *halt;       // the solve loop's halt flag (nullable): the call does nothing when set
    int n_pre, n_post, n_cycles, n_coarse;
};

template <typename T>
struct Lv {
    T *x, *f, *d;
    int nx, ny, nz, n;
    unsigned long long mx, mxy;  // ceil(2^32 / nx), ceil(2^32 / (nx*ny))
    int hx;                      // cells of one colour per row, at most: ceil(nx / 2)
    unsigned long long mh, mhy;  // ceil(2^32 / hx), ceil(2^32 / (hx*ny))
    T h2, ih2;
};

// Division magics of a level for the host: ceil(2^32 / v).
inline unsigned long long div_magic(unsigned v) { return (0x100000000ull + v - 1) / v; }

// Exact quotient e / d for e * d < 2^32, with m = ceil(2^32 / d): the error
// of e * m / 2^32 is below e / 2^32 < 1/d, too small to reach the next integer.
__device__ __forceinline__ int qdiv(int e, unsigned long long m) {
    return (int)(((unsigned long long)(unsigned)e * m) >> 32);
}

template <typename T>
__device__ __forceinline__ void cell_ijk(const Lv<T> &L, int e, int &i, int &j, int &k) {
    k = qdiv(e, L.mxy);
    const int r = e - k * L.nx * L.ny;
    j = qdiv(r, L.mx);
    i = r - j * L.nx;
}

template <typename T>
__device__ __forceinline__ T nb_sum(const T *x, int i, int j, int k, int nx, int ny, int nz) {
    const int p = (k * ny + j) * nx + i;
    const T xm = i > 0 ? x[p - 1] : T(0);
    const T xp = i < nx - 1 ? x[p + 1] : T(0);
    const T ym = j > 0 ? x[p - nx] : T(0);
    const T yp = j < ny - 1 ? x[p + nx] : T(0);
    const T zm = k > 0 ? x[p - nx * ny] : T(0);
    const T zp = k < nz - 1 ? x[p + nx * ny] : T(0);
    return (xm + xp) + (ym + yp) + (zm + zp);
}

// The three relaxation paths below (one wave, cells in registers, slots in
// turn) are chosen by level size and thread count; each evaluates
// ((x-neighbour pair) + (y pair) + (z pair) - h^2 f) / d with h^2 f rounded
// on its own (no fused multiply-add) and the quotient correctly rounded (by
// a division, or, where a cell's diagonal stays in registers over the passes,
// from its correctly rounded reciprocal with one correction step: rb::
// div_small), so every path, for any thread count, gives the same value bit
// for bit.

// Red-black half-sweep of colour `col` over slots first, first + step, ...
// (slot m of row (j, k) is cell i = 2m + ((col + j + k) mod 2)).
template <typename T>
__device__ __forceinline__ void half_sweep(const Lv<T> &L, int col, int first, int step) {
#pragma clang fp contract(off)
    const int slots = L.hx * L.ny * L.nz;
    for (int s = first; s < slots; s += step) {
        const int k = qdiv(s, L.mhy);
        const int r = s - k * L.hx * L.ny;
        const int j = qdiv(r, L.mh);
        const int i = 2 * (r - j * L.hx) + ((col + j + k) & 1);
        if (i >= L.nx) continue;
        const int e = (k * L.ny + j) * L.nx + i;
        const T d = L.d[e];
        if (d == T(0)) continue;
        L.x[e] = (nb_sum(L.x, i, j, k, L.nx, L.ny, L.nz) - L.h2 * L.f[e]) / d;
    }
}

// Levels with at most 64 cells of one colour are relaxed by the first wave
// alone, each lane owning at most one cell per colour: its index, neighbour
// validity, diagonal and h^2 f stay in registers for all passes.  A wave's LDS
// accesses complete in order, so its half-sweeps need no workgroup barrier
// between them (the other waves wait once at the end).
constexpr int WAVE_SLOTS = 64;

template <typename T>
__device__ __forceinline__ void smooth_wave(const Lv<T> &L, int passes) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x;
    const int nxy = L.nx * L.ny;
    int e[2] = {-1, -1};
    unsigned nb[2] = {0u, 0u};  // valid neighbours: -x, +x, -y, +y, -z, +z
    T dg[2] = {T(1), T(1)}, yr[2] = {T(1), T(1)}, rhs[2] = {T(0), T(0)};
#pragma unroll
    for (int col = 0; col < 2; col++) {
        if (lane >= L.hx * L.ny * L.nz) continue;
        const int k = qdiv(lane, L.mhy);
        const int r = lane - k * L.hx * L.ny;
        const int j = qdiv(r, L.mh);
        const int i = 2 * (r - j * L.hx) + ((col + j + k) & 1);
        if (i >= L.nx) continue;
        const int c = (k * L.ny + j) * L.nx + i;
        if (L.d[c] == T(0)) continue;
        e[col] = c;
        dg[col] = L.d[c];
        yr[col] = T(1) / dg[col];
        rhs[col] = L.h2 * L.f[c];
        nb[col] = (unsigned)(i > 0) | (unsigned)(i < L.nx - 1) << 1 | (unsigned)(j > 0) << 2 |
                  (unsigned)(j < L.ny - 1) << 3 | (unsigned)(k > 0) << 4 | (unsigned)(k < L.nz - 1) << 5;
    }
    for (int p = 0; p < passes; p++)
#pragma unroll
        for (int col = 0; col < 2; col++) {
            const int c = e[col];
            if (c >= 0) {
                const unsigned m = nb[col];
                const T *x = L.x;
                const T xm = (m & 1u) ? x[c - 1] : T(0);
                const T xp = (m & 2u) ? x[c + 1] : T(0);
                const T ym = (m & 4u) ? x[c - L.nx] : T(0);
                const T yp = (m & 8u) ? x[c + L.nx] : T(0);
                const T zm = (m & 16u) ? x[c - nxy] : T(0);
                const T zp = (m & 32u) ? x[c + nxy] : T(0);
                L.x[c] = rb::div_small<T>(((xm + xp) + (ym + yp) + (zm + zp)) - rhs[col], dg[col], yr[col]);
            }
            // keep the next half-sweep's LDS reads behind this one's writes
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
}

// Levels with at most two cells of one colour per thread: each thread keeps
// its cells' index, neighbour validity, diagonal and f in registers for all
// passes of the call (the same expression as half_sweep).
template <typename T, int NTH>
__device__ void smooth_regs(const Lv<T> &L, int passes) {
#pragma clang fp contract(off)
    const int slots = L.hx * L.ny * L.nz;
    const int nxy = L.nx * L.ny;
    int e[2][2];
    unsigned nb[2][2];
    T dg[2][2], yr[2][2], fv[2][2];
#pragma unroll
    for (int col = 0; col < 2; col++)
#pragma unroll
        for (int u = 0; u < 2; u++) {
            e[col][u] = -1;
            nb[col][u] = 0u;
            dg[col][u] = T(1);
            yr[col][u] = T(1);
            fv[col][u] = T(0);
            const int s = threadIdx.x + u * NTH;
            if (s >= slots) continue;
            const int k = qdiv(s, L.mhy);
            const int r = s - k * L.hx * L.ny;
            const int j = qdiv(r, L.mh);
            const int i = 2 * (r - j * L.hx) + ((col + j + k) & 1);
            if (i >= L.nx) continue;
            const int c = (k * L.ny + j) * L.nx + i;
            const T d = L.d[c];
            if (d == T(0)) continue;
            e[col][u] = c;
            dg[col][u] = d;
            yr[col][u] = T(1) / d;
            fv[col][u] = L.f[c];
            nb[col][u] = (unsigned)(i > 0) | (unsigned)(i < L.nx - 1) << 1 | (unsigned)(j > 0) << 2 |
                         (unsigned)(j < L.ny - 1) << 3 | (unsigned)(k > 0) << 4 | (unsigned)(k < L.nz - 1) << 5;
        }
    for (int p = 0; p < passes; p++)
#pragma unroll
        for (int col = 0; col < 2; col++) {
#pragma unroll
            for (int u = 0; u < 2; u++) {
                const int c = e[col][u];
                if (c < 0) continue;
                const unsigned m = nb[col][u];
                const T *x = L.x;
                const T xm = (m & 1u) ? x[c - 1] : T(0);
                const T xp = (m & 2u) ? x[c + 1] : T(0);
                const T ym = (m & 4u) ? x[c - L.nx] : T(0);
                const T yp = (m & 8u) ? x[c + L.nx] : T(0);
                const T zm = (m & 16u) ? x[c - nxy] : T(0);
                const T zp = (m & 32u) ? x[c + nxy] : T(0);
                L.x[c] = rb::div_small<T>(((xm + xp) + (ym + yp) + (zm + zp)) - L.h2 * fv[col][u], dg[col][u],
                                          yr[col][u]);
            }
            __syncthreads();
        }
}

// Red-black passes; each half-sweep visits only the cells of its colour.
// WAVE: a level of at most WAVE_SLOTS slots per colour runs on one wave with
// no block barrier (levels in LDS only; with levels in global memory every
// half-sweep ends at a block barrier).
template <typename T, int NTH, bool WAVE = true>
__device__ void smooth(const Lv<T> &L, int passes) {
    const int slots = L.hx * L.ny * L.nz;
    if (WAVE && slots <= WAVE_SLOTS) {
        if (threadIdx.x < 64) smooth_wave(L, passes);
        __syncthreads();
        return;
    }
    if (slots <= 2 * NTH) {
        smooth_regs<T, NTH>(L, passes);
        return;
    }
    for (int p = 0; p < passes; p++)
        for (int col = 0; col < 2; col++) {
            half_sweep(L, col, threadIdx.x, NTH);
            __syncthreads();
        }
}

// f_c = -(1/8) sum over active children of (L x - f); x_c = 0.
template <typename T, int NTH>
__device__ void restrict_to(const Lv<T> &L, const Lv<T> &C) {
    for (int E = threadIdx.x; E < C.n; E += NTH) {
        int I, J, K;
        cell_ijk(C, E, I, J, K);
        T s = T(0);
        if (C.d[E] != T(0)) {
#pragma unroll
            for (int c = 0; c < 8; c++) {
                const int i = 2 * I + (c & 1), j = 2 * J + ((c >> 1) & 1), k = 2 * K + (c >> 2);
                const int p = (k * L.ny + j) * L.nx + i;
                const T d = L.d[p];
                if (d != T(0)) s += (nb_sum(L.x, i, j, k, L.nx, L.ny, L.nz) - d * L.x[p]) * L.ih2 - L.f[p];
            }
            s = -s / T(8);
        }
        C.f[E] = s;
        C.x[E] = T(0);
    }
    __syncthreads();
}

// x += P2(x_c) on active cells (weights 3/4, 1/4 per axis; 0 off the box).
template <typename T, int NTH>
__device__ void prolong_from(const Lv<T> &L, const Lv<T> &C) {
    const T w[2] = {T(0.75), T(0.25)};
    for (int e = threadIdx.x; e < L.n; e += NTH) {
        if (L.d[e] == T(0)) continue;
        int i, j, k;
        cell_ijk(L, e, i, j, k);
        const int I = i >> 1, J = j >> 1, K = k >> 1;
        const int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
        T s = T(0);
#pragma unroll
        for (int c = 0; c < 2; c++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int a = 0; a < 2; a++) {
                    const int ci = I + a * sx, cj = J + b * sy, ck = K + c * sz;
                    T v = T(0);
                    if (ci >= 0 && ci < C.nx && cj >= 0 && cj < C.ny && ck >= 0 && ck < C.nz)
                        v = C.x[(ck * C.ny + cj) * C.nx + ci];
                    s += w[a] * w[b] * w[c] * v;
                }
        L.x[e] += s;
    }
    __syncthreads();
}

// One call MG(ls) for the levels held in S, all resident at `sm`: in LDS
// (WAVE: the one-wave path relies on a wave's in-order LDS accesses), or in
// a global-memory area of the block's own (!WAVE: block barriers only); f0 is
// level ls's right-hand side and x0 its iterate (in/out), started from zero
// unless load_x.  Called by all NTH threads of a block.
template <typename T, int NTH, bool WAVE = true>
__device__ void small_tail(T *sm, const SmallLevels<T> &S, const T *f0, T *x0, bool load_x) {
    // level descriptors live in LDS (dynamic indexing without private memory)
    __shared__ int s_nx[MAXS], s_ny[MAXS], s_nz[MAXS], s_off[MAXS];
    __shared__ unsigned long long s_mx[MAXS], s_mxy[MAXS], s_mh[MAXS], s_mhy[MAXS];
    __shared__ T s_h2[MAXS], s_ih2[MAXS];
    __shared__ const T *s_d[MAXS];
    if (threadIdx.x < (unsigned)S.n) {
        const int l = threadIdx.x;
        s_nx[l] = S.nx[l];
        s_ny[l] = S.ny[l];
        s_nz[l] = S.nz[l];
        s_off[l] = S.off[l];
        s_mx[l] = S.mx[l];
        s_mxy[l] = S.mxy[l];
        s_mh[l] = S.mh[l];
        s_mhy[l] = S.mhy[l];
        s_h2[l] = S.h2[l];
        s_ih2[l] = S.ih2[l];
        s_d[l] = S.d[l];
    }
    __syncthreads();
    auto level = [&](int l) {
        Lv<T> v;
        v.nx = s_nx[l];
        v.ny = s_ny[l];
        v.nz = s_nz[l];
        v.n = v.nx * v.ny * v.nz;
        v.mx = s_mx[l];
        v.mxy = s_mxy[l];
        v.hx = (v.nx + 1) >> 1;
        v.mh = s_mh[l];
        v.mhy = s_mhy[l];
        v.x = sm + s_off[l];
        v.f = v.x + v.n;
        v.d = v.f + v.n;
        v.h2 = s_h2[l];
        v.ih2 = s_ih2[l];
        return v;
    };
    // Copy-in: every level's cells as one flat range, U elements per thread
    // loaded before any is stored, so that their global loads overlap.
    auto cells = [&](int l) { return s_nx[l] * s_ny[l] * s_nz[l]; };
    int tot = 0;
    for (int l = 0; l < S.n; l++) tot += cells(l);
    constexpr int U = 8;
    for (int q0 = threadIdx.x; q0 < tot; q0 += U * NTH) {
        T dv[U], fv[U], xv[U];
        int lv[U], ev[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            int l = 0, e = q0 + u * NTH;
            lv[u] = -1;
            if (e >= tot) continue;
            while (e >= cells(l)) {
                e -= cells(l);
                l++;
            }
            lv[u] = l;
            ev[u] = e;
            dv[u] = s_d[l][e];
            fv[u] = l == 0 ? f0[e] : T(0);
            xv[u] = (l == 0 && load_x) ? x0[e] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            if (lv[u] < 0) continue;
            const Lv<T> v = level(lv[u]);
            v.d[ev[u]] = dv[u];
            v.x[ev[u]] = xv[u];
            if (lv[u] == 0) v.f[ev[u]] = fv[u];
        }
    }
    __syncthreads();
    // iterative form of the recursion MG(l): pre-smooth, restrict, N_cycles x
    // MG(l+1) from zero, prolong, post-smooth; the deepest level is relaxed.
    // visits: 3 bits per level (N_cycles <= 4).
    const int last = S.n - 1;
    unsigned visits = 0;
    int l = 0;
    bool down = true;
    while (true) {
        if (down) {
            if (l == last) {
                smooth<T, NTH, WAVE>(level(l), S.n_coarse);
                down = false;
                continue;
            }
            smooth<T, NTH, WAVE>(level(l), S.n_pre);
            restrict_to<T, NTH>(level(l), level(l + 1));
            visits &= ~(7u << (3 * (l + 1)));
            l++;
            continue;
        }
        if (l == 0) break;
        const unsigned vc = ((visits >> (3 * l)) & 7u) + 1u;
        visits = (visits & ~(7u << (3 * l))) | (vc << (3 * l));
        if ((int)vc < S.n_cycles) {
            down = true;
            continue;
        }
        prolong_from<T, NTH>(level(l - 1), level(l));
        smooth<T, NTH, WAVE>(level(l - 1), S.n_post);
        l--;
    }
    const Lv<T> top = level(0);
    for (int e = threadIdx.x; e < top.n; e += NTH) x0[e] = top.x[e];
    __syncthreads();
}

}  // namespace small
}  // namespace mg
