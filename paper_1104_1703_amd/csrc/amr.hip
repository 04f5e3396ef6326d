// One-way interface between nested levels (AMR; Sec. 3 "one-way interface",
// Sec. 5.1 accuracy tests, Fig. "force-ramses"): Dirichlet values of a
// refined patch from the next coarser level's potential, and the gradient of
// the potential by the 5-point difference with the values beyond a level's
// boundary taken from the coarser level.  Both interpolate the coarser
// cell-centred potential linearly (trilinear between its cell centres).
//
// A level is a box array (nz, ny, nx) of cells of width h, lower corner at
// origin (x0, y0, z0): cell (i, j, k) has its centre at origin + (idx + 1/2) h.
// Multiplies and adds are kept separate (no fused multiply-add) so every
// value is the correctly rounded result of the defining expression.
#include <math.h>

#include "mg_core.h"

#pragma clang fp contract(off)

namespace mg {
namespace {

struct Coarse {
    const double *phi;
    int nx, ny, nz;
    double h, ox, oy, oz;
};

// Trilinear interpolation at (x, y, z); NaN when the 8 surrounding centres
// are not all inside the array (the host validates the geometry first).
__device__ double interp(const Coarse &C, double x, double y, double z) {
    const double sx = (x - C.ox) / C.h - 0.5, sy = (y - C.oy) / C.h - 0.5, sz = (z - C.oz) / C.h - 0.5;
    const double bx = floor(sx), by = floor(sy), bz = floor(sz);
    const int I = (int)bx, J = (int)by, K = (int)bz;
    if (I < 0 || J < 0 || K < 0 || I + 1 >= C.nx || J + 1 >= C.ny || K + 1 >= C.nz) return NAN;
    const double tx = sx - bx, ty = sy - by, tz = sz - bz;
    const double wx[2] = {1.0 - tx, tx}, wy[2] = {1.0 - ty, ty}, wz[2] = {1.0 - tz, tz};
    double out = 0.0;
    for (int c = 0; c < 2; c++)
        for (int b = 0; b < 2; b++)
            for (int a = 0; a < 2; a++) {
                const double w = wz[c] * wy[b] * wx[a];
                out = out + w * C.phi[((size_t)(K + c) * C.ny + (J + b)) * C.nx + (I + a)];
            }
    return out;
}

// B on a patch whose outer layer is its boundary: interior cells take the
// interpolated coarse potential at their centre; a frame cell face-adjacent
// to one interior cell takes 2 g - B_i (g: the interpolated potential at the
// shared face's centre) so the face value (B_i + B_j) / 2 the solver reads is
// g; edge and corner frame cells take 0.
__global__ void k_amr_dirichlet(Coarse C, int nx, int ny, int nz, double h, double ox, double oy, double oz,
                                double *__restrict__ B) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = (size_t)nx * ny * nz;
    if (e >= n) return;
    const int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((size_t)nx * ny));
    const bool ix = i >= 1 && i <= nx - 2, iy = j >= 1 && j <= ny - 2, iz = k >= 1 && k <= nz - 2;
    auto cx = [&](int q) { return ox + (q + 0.5) * h; };
    auto cy = [&](int q) { return oy + (q + 0.5) * h; };
    auto cz = [&](int q) { return oz + (q + 0.5) * h; };
    double v = 0.0;
    if (ix && iy && iz) {
        v = interp(C, cx(i), cy(j), cz(k));
    } else if (iy && iz && (i == 0 || i == nx - 1)) {
        const int a = i == 0 ? 1 : nx - 2;
        const double g = interp(C, 0.5 * (cx(i) + cx(a)), cy(j), cz(k));
        v = 2.0 * g - interp(C, cx(a), cy(j), cz(k));
    } else if (ix && iz && (j == 0 || j == ny - 1)) {
        const int a = j == 0 ? 1 : ny - 2;
        const double g = interp(C, cx(i), 0.5 * (cy(j) + cy(a)), cz(k));
        v = 2.0 * g - interp(C, cx(i), cy(a), cz(k));
    } else if (ix && iy && (k == 0 || k == nz - 1)) {
        const int a = k == 0 ? 1 : nz - 2;
        const double g = interp(C, cx(i), cy(j), 0.5 * (cz(k) + cz(a)));
        v = 2.0 * g - interp(C, cx(i), cy(j), cz(a));
    }
    B[e] = v;
}

// d phi / d x (and y, z) = (4/3) (phi[+1] - phi[-1]) / (2 h) - (1/3) (phi[+2] - phi[-2]) / (4 h)
// on active cells; a value at a cell that is not an active cell of this level
// comes from the coarser level at that cell's centre, or, with no coarser
// level, from the Dirichlet field bnd inside the array (NaN beyond).
// Output: three (nz, ny, nx) components x, y, z; inactive cells get 0.
__global__ void k_amr_grad5(const double *__restrict__ phi, const int8_t *__restrict__ mask, int nx, int ny, int nz,
                            double h, double ox, double oy, double oz, Coarse C, const double *__restrict__ bnd,
                            double *__restrict__ grad) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t n = (size_t)nx * ny * nz;
    if (e >= n) return;
    if (mask[e] != 1) {
        grad[e] = 0.0;
        grad[n + e] = 0.0;
        grad[2 * n + e] = 0.0;
        return;
    }
    const int i = (int)(e % nx), j = (int)((e / nx) % ny), k = (int)(e / ((size_t)nx * ny));
    auto value = [&](int a, int b, int c) -> double {
        const bool inside = a >= 0 && a < nx && b >= 0 && b < ny && c >= 0 && c < nz;
        const size_t q = inside ? ((size_t)c * ny + b) * nx + a : 0;
        if (inside && mask[q] == 1) return phi[q];
        if (C.phi) return interp(C, ox + (a + 0.5) * h, oy + (b + 0.5) * h, oz + (c + 0.5) * h);
        return inside && bnd ? bnd[q] : NAN;
    };
    for (int ax = 0; ax < 3; ax++) {
        const int dx = ax == 0, dy = ax == 1, dz = ax == 2;
        const double p1 = value(i + dx, j + dy, k + dz), m1 = value(i - dx, j - dy, k - dz);
        const double p2 = value(i + 2 * dx, j + 2 * dy, k + 2 * dz), m2 = value(i - 2 * dx, j - 2 * dy, k - 2 * dz);
        grad[ax * n + e] = (4.0 / 3.0) * (p1 - m1) / (2.0 * h) - (1.0 / 3.0) * (p2 - m2) / (4.0 * h);
    }
}

// The coarser array must hold the 8-centre stencil of every point in the
// box [lo, hi] (per axis).
bool covers(const Coarse &C, const double lo[3], const double hi[3]) {
    const double o[3] = {C.ox, C.oy, C.oz};
    const int n[3] = {C.nx, C.ny, C.nz};
    for (int a = 0; a < 3; a++) {
        const double s0 = (lo[a] - o[a]) / C.h - 0.5, s1 = (hi[a] - o[a]) / C.h - 0.5;
        if (!(s0 >= 0.0) || !(floor(s1) + 1.0 <= n[a] - 1.0)) return false;
    }
    return true;
}

bool dims_ok(int nx, int ny, int nz) { return nx >= 3 && ny >= 3 && nz >= 3; }

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" {

mg_status mg_amr_dirichlet(const double *phi_c_dev, int32_t cnx, int32_t cny, int32_t cnz, double hc,
                           const double *origin_c, int32_t nx, int32_t ny, int32_t nz, double hf,
                           const double *origin_f, double *b_dev, void *stream) {
    set_error("");
    if (!phi_c_dev || !origin_c || !origin_f || !b_dev || !dims_ok(cnx, cny, cnz) || !dims_ok(nx, ny, nz) ||
        !(hc > 0) || !(hf > 0)) {
        set_error("invalid mg_amr_dirichlet arguments");
        return MG_ERR_ARG;
    }
    const Coarse C{phi_c_dev, cnx, cny, cnz, hc, origin_c[0], origin_c[1], origin_c[2]};
    // points used: interior centres and the faces of the interior block
    const double lo[3] = {origin_f[0] + hf, origin_f[1] + hf, origin_f[2] + hf};
    const double hi[3] = {origin_f[0] + (nx - 1) * hf, origin_f[1] + (ny - 1) * hf, origin_f[2] + (nz - 1) * hf};
    if (!covers(C, lo, hi)) {
        set_error("the coarser level does not cover the patch boundary");
        return MG_ERR_ARG;
    }
    const size_t n = (size_t)nx * ny * nz;
    k_amr_dirichlet<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(C, nx, ny, nz, hf, origin_f[0],
                                                                                  origin_f[1], origin_f[2], b_dev);
    return hip_ok(hipGetLastError(), "k_amr_dirichlet") ? MG_OK : MG_ERR_HIP;
}

mg_status mg_amr_grad5(const double *phi_dev, const int8_t *mask_dev, int32_t nx, int32_t ny, int32_t nz, double h,
                       const double *origin, const double *phi_c_dev, int32_t cnx, int32_t cny, int32_t cnz,
                       double hc, const double *origin_c, const double *bnd_dev, double *grad_dev, void *stream) {
    set_error("");
    if (!phi_dev || !mask_dev || !origin || !grad_dev || !dims_ok(nx, ny, nz) || !(h > 0)) {
        set_error("invalid mg_amr_grad5 arguments");
        return MG_ERR_ARG;
    }
    Coarse C{nullptr, 0, 0, 0, 1.0, 0.0, 0.0, 0.0};
    if (phi_c_dev) {
        if (!origin_c || !dims_ok(cnx, cny, cnz) || !(hc > 0)) {
            set_error("invalid coarser level in mg_amr_grad5");
            return MG_ERR_ARG;
        }
        C = Coarse{phi_c_dev, cnx, cny, cnz, hc, origin_c[0], origin_c[1], origin_c[2]};
        // values may be needed at any cell centre up to two cells beyond the array
        const double lo[3] = {origin[0] - 1.5 * h, origin[1] - 1.5 * h, origin[2] - 1.5 * h};
        const double hi[3] = {origin[0] + (nx + 1.5) * h, origin[1] + (ny + 1.5) * h, origin[2] + (nz + 1.5) * h};
        if (!covers(C, lo, hi)) {
            set_error("the coarser level does not cover the level and its 2-cell margin");
            return MG_ERR_ARG;
        }
    }
    const size_t n = (size_t)nx * ny * nz;
    k_amr_grad5<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        phi_dev, mask_dev, nx, ny, nz, h, origin[0], origin[1], origin[2], C, bnd_dev, grad_dev);
    return hip_ok(hipGetLastError(), "k_amr_grad5") ? MG_OK : MG_ERR_HIP;
}

}  // extern "C"
