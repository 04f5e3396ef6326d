// Kernels of the learned initial guess: a 3D U-Net whose convolutions are
// implicit GEMMs on the gfx950 BF16 matrix cores (v_mfma_f32_16x16x32_bf16),
// BF16 storage and FP32 accumulation.  Tensors are channels-last (NDHWC):
// element (n, z, y, x, c) at ((((n*D + z)*H + y)*W + x)*C + c).
//
// Convolution (3x3x3, zero padding, stride 1) as a GEMM: M = voxels,
// N = output channels, K = 27 taps x input channels.  A wave owns 4 x 16
// voxels by NTC x 16 output channels.  At each K step of 32, lane l supplies
// row (l mod 16) of A and column (l mod 16) of B as 8 consecutive K entries
// starting at 8*(l div 16); with channels-last tensors and [tap][co][ci]
// weights both are single 16-byte reads (A from a halo tile in LDS, B from
// global memory).  The input may be the channel concatenation of a tensor
// read at half resolution (nearest up-sampling, resolved while the tile is
// staged) and a full-resolution tensor.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mg.h"
#include "mg_core.h"
#include "nn_core.h"

namespace mg {
namespace nn {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NTH = 256;

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int j = 0; j < 8; j++) z[j] = (bf16)0.0f;
    return z;
}

__device__ __forceinline__ f32x4 mfma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------ conv fwd, LDS tiles
// out = [ReLU](conv3x3x3(concat(up2?(ina), inb)) + bias) as an implicit GEMM
// (M = voxels, N = output channels, K = 27 taps x input channels), organised
// around LDS: a block owns a 16 x 4 x 4 tile of output voxels of one sample
// and, for each chunk of CK input channels, stages the 18 x 6 x 6 halo of its
// input in LDS (zeros outside the box, nearest up-sampling and the skip
// concatenation resolved while staging).  The tap loop then reads every A
// fragment from LDS at a uniform tap offset, with no bounds tests.  Wave w
// computes z-plane w of the tile; its fragment mt is row y = mt, lane row r
// the voxel x = r.  A voxel's LDS row is CK + 8 channels long (an odd number
// of 16-byte bank groups), so the 16 x-consecutive rows of a fragment fall in
// 16 distinct bank groups.  A chunk holding only 16 input channels (CK = 16,
// or with HALF the last chunk when C_in = 32 q + 16) takes two taps per K step
// of 32 (lane groups 0, 1: tap 2p; 2, 3: tap 2p + 1) instead of padding K
// with zeros.
constexpr int TX = 16, TY = 4, TZ = 4;
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HV = HX * HY * HZ;

template <int CK, int NTC, bool HALF = false>
__global__ __launch_bounds__(NTH) void k_conv_tile(const bf16 *__restrict__ ina, int ca, int upa,
                                                   const bf16 *__restrict__ inb, int cb, const bf16 *__restrict__ wt,
                                                   const float *__restrict__ bias, bf16 *__restrict__ out, int cout,
                                                   int relu, int D, int H, int W, int ntx, int nty, int ntz,
                                                   int nblk) {
    constexpr int CKP = CK + 8;
    constexpr int MT = 4;
    static_assert(MT == TY && NTH / 64 == TZ && TX == 16, "a wave owns the 16 x 4 voxels of one tile plane");
    __shared__ __attribute__((aligned(16))) bf16 tile[HV * CKP];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, grp = lane >> 4;
    // the 8 XCDs take contiguous runs of tiles, so neighbouring halos share an L2
    int b = blockIdx.x;
    if ((nblk & 7) == 0) b = (b & 7) * (nblk >> 3) + (b >> 3);
    const int tx = b % ntx;
    int t = b / ntx;
    const int ty = t % nty;
    t /= nty;
    const int tz = t % ntz;
    const int n = t / ntz;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
    const int co_base = blockIdx.y * NTC * 16;
    const int cin = ca + cb;
    const int Dc = D >> 1, Hc = H >> 1, Wc = W >> 1;
    int hb[MT];
#pragma unroll
    for (int mt = 0; mt < MT; mt++) hb[mt] = ((wave + 1) * HY + mt + 1) * HX + row + 1;
    f32x4 acc[MT][NTC];
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int nt = 0; nt < NTC; nt++) acc[mt][nt] = f32x4{0.f, 0.f, 0.f, 0.f};

    // Staging: thread t copies the 16-byte piece `sub` of voxels t / SUB,
    // t / SUB + VPT, ... of the halo tile, its (row, x) stepped by VPT voxels
    // in mixed radix (no divisions in the loop).
    constexpr int SUB = CK / 8, VPT = NTH / SUB;
    const int sub = threadIdx.x % SUB, hv0 = threadIdx.x / SUB;
    // base pointers of the halo's 36 (z, y) source rows at x = 0, per input
    // (null outside the box), built once per block: an element's address is
    // then its row base plus x times the voxel stride
    __shared__ const bf16 *rowb[2][HZ * HY];
    if (threadIdx.x < 2 * HZ * HY) {
        const int src = threadIdx.x / (HZ * HY), r = threadIdx.x % (HZ * HY);
        const int gz = z0 - 1 + r / HY, gy = y0 - 1 + r % HY;
        const bf16 *bp = nullptr;
        if ((unsigned)gz < (unsigned)D && (unsigned)gy < (unsigned)H) {
            if (src == 0)
                bp = upa ? ina + ((((size_t)n * Dc + (gz >> 1)) * Hc + (gy >> 1)) * Wc) * ca
                         : ina + ((((size_t)n * D + gz) * H + gy) * W) * ca;
            else if (inb)
                bp = inb + ((((size_t)n * D + gz) * H + gy) * W) * cb;
        }
        rowb[src][r] = bp;
    }
    // A fragments: LDS element offset of tap (dz, dy, dx) is toff * CKP with
    // toff = ((dz - 1) HY + dy - 1) HX + dx - 1 >= -TMIN; bases shifted by
    // TMIN keep every offset a non-negative constant
    constexpr int TMIN = HY * HX + HX + 1;
    const bf16 *tb[MT];
#pragma unroll
    for (int mt = 0; mt < MT; mt++) tb[mt] = tile + (hb[mt] - TMIN) * CKP;
    // weights [tap][co][ci]: a uniform per-tap base and this lane's offset
    const size_t wtap = (size_t)cout * cin;
    for (int c0 = 0; c0 < cin; c0 += CK) {
        __syncthreads();
        {
            const int c = c0 + sub * 8;  // this thread's 8 channels: all of a or all of b (8 | ca)
            const bool cok = c < cin, isa = c < ca;
            const int coff = isa ? c : c - ca, cs = isa ? ca : cb, sh = (isa && upa) ? 1 : 0;
            const bf16 *const *rb = rowb[isa ? 0 : 1];
            // voxel hv = row hr (z-major over (z, y)) x HX + hx, stepped by VPT
            constexpr int SDR = VPT / HX, SDX2 = VPT % HX;
            int hv = hv0, hx = hv0 % HX, hr = hv0 / HX;
#pragma unroll
            for (int k = 0; k < (HV + VPT - 1) / VPT; k++) {
                if (hv < HV) {
                    const int gx = x0 - 1 + hx;
                    const bf16 *bp = rb[hr];
                    bf16x8 v = zero8();
                    if (cok && bp && (unsigned)gx < (unsigned)W)  // x < 2^24, channels < 2^24
                        v = *(const bf16x8 *)(bp + (__umul24((unsigned)(gx >> sh), (unsigned)cs) + coff));
                    *(bf16x8 *)(tile + hv * CKP + sub * 8) = v;
                }
                hv += VPT;
                hx += SDX2;
                hr += SDR;
                if (hx >= HX) {
                    hx -= HX;
                    hr++;
                }
            }
        }
        __syncthreads();
        if (CK == 32 && (!HALF || cin - c0 >= 32)) {
            const int cw = c0 + grp * 8;  // this lane's 8 K entries: channels cw .. cw + 7 of one tap
            unsigned wl[NTC];  // byte offsets within a tap's weights
#pragma unroll
            for (int nt = 0; nt < NTC; nt++) wl[nt] = (unsigned)(((co_base + nt * 16 + row) * cin + cw) * 2);
#pragma unroll 1
            for (int tzy = 0; tzy < 9; ++tzy) {  // (dz, dy) rows of taps; the 3 dx taps unrolled
                const int rowoff = ((tzy / 3 - 1) * HY + tzy % 3 - 1) * HX;  // uniform
                // the row's 3 x MT A fragments and 3 x NTC B fragments are all
                // read before its matrix products
                bf16x8 afr[3][MT], bfr[3][NTC];
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const char *wb = (const char *)(wt + (tzy * 3 + dx) * wtap);  // uniform
#pragma unroll
                    for (int nt = 0; nt < NTC; nt++) bfr[dx][nt] = *(const bf16x8 *)(wb + wl[nt]);
                }
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                    for (int mt = 0; mt < MT; mt++)
                        afr[dx][mt] = *(const bf16x8 *)(tb[mt] + (rowoff + TMIN - 1 + dx) * CKP + grp * 8);
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                    for (int mt = 0; mt < MT; mt++)
#pragma unroll
                        for (int nt = 0; nt < NTC; nt++) acc[mt][nt] = mfma(afr[dx][mt], bfr[dx][nt], acc[mt][nt]);
                // schedule: the row's weight loads, its LDS reads, then its matrix products
                __builtin_amdgcn_sched_group_barrier(0x020, 3 * NTC, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 3 * MT, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, 3 * MT * NTC, 0);
            }
        } else if constexpr (CK == 16 || HALF) {
            // 16 channels per tap: one K step of 32 covers taps 2p (lane groups 0, 1) and 2p + 1 (2, 3)
            const int half = grp >> 1, cl = (grp & 1) * 8, cw = c0 + cl;
            const bool cok = cw < cin;
            unsigned wl[NTC];  // byte offsets within tap 2p's weights (this lane's tap is 2p + half)
#pragma unroll
            for (int nt = 0; nt < NTC; nt++)
                wl[nt] = (unsigned)((half * (int)wtap + (co_base + nt * 16 + row) * cin + cw) * 2);
            const bf16 *tc[MT];
#pragma unroll
            for (int mt = 0; mt < MT; mt++) tc[mt] = tb[mt] + TMIN * CKP + cl;
#pragma unroll 2
            for (int p = 0; p < 14; ++p) {
                const int t0 = 2 * p, t1 = 2 * p + 1;  // uniform; this lane's tap is t0 + half
                const int o0 = ((t0 / 9 - 1) * HY + (t0 / 3) % 3 - 1) * HX + t0 % 3 - 1;
                const int o1 = t1 < 27 ? ((t1 / 9 - 1) * HY + (t1 / 3) % 3 - 1) * HX + t1 % 3 - 1 : 0;
                const bool tok = cok && (t1 < 27 || !half);
                const int toff = (half ? o1 : o0) * CKP;
                const char *wb = (const char *)(wt + t0 * wtap);  // uniform
                bf16x8 bfr[NTC];
#pragma unroll
                for (int nt = 0; nt < NTC; nt++) bfr[nt] = tok ? *(const bf16x8 *)(wb + wl[nt]) : zero8();
#pragma unroll
                for (int mt = 0; mt < MT; mt++) {
                    const bf16x8 afr = tok ? *(const bf16x8 *)(tc[mt] + toff) : zero8();
#pragma unroll
                    for (int nt = 0; nt < NTC; nt++) acc[mt][nt] = mfma(afr, bfr[nt], acc[mt][nt]);
                }
            }
        }
    }
    // lane l holds D[4 (l div 16) + r][l mod 16]: voxel x = 4 grp + r of row y = mt, channel row
    const int z = z0 + wave;
    // this lane's first output (x0 + 4 grp, y0, z, channel co_base + row)
    bf16 *ob = out + ((((size_t)n * D + z) * H + y0) * W + x0 + grp * 4) * cout + co_base + row;
#pragma unroll
    for (int mt = 0; mt < MT; mt++)
#pragma unroll
        for (int nt = 0; nt < NTC; nt++) {
            const int co = co_base + nt * 16 + row;
            const float bv = bias ? bias[co] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int x = x0 + grp * 4 + r, y = y0 + mt;
                if (x < W && y < H && z < D) {
                    float val = acc[mt][nt][r] + bv;
                    if (relu) val = fmaxf(val, 0.f);
                    ob[(size_t)(mt * W + r) * cout + nt * 16] = (bf16)val;
                }
            }
        }
}

// -------------------------------------------------------------- conv bwd W
// dW[tap][co][ci] += sum_v dout[v][co] * X[v shifted by tap][ci] (X the
// possibly concatenated, possibly upsampled input), dbias[co] += sum_v dout.
// GEMM per tap: M = co, N = ci, K = voxels.  A block takes one tap, 64
// output channels (one 16-channel tile per wave) and a chunk of voxels; 32
// voxels at a time are staged in LDS (dout rows and shifted input rows,
// contiguous loads), then read back transposed as MFMA fragments.  Partial
// sums go to global FP32 with atomics.
constexpr int BW_KV = 32;

template <int NCI>  // input-channel tiles of 16 (cin = 16 * NCI)
__global__ __launch_bounds__(NTH) void k_conv_bwd_w(const bf16 *__restrict__ dout, int cout,
                                                     const bf16 *__restrict__ ina, int ca, int upa,
                                                     const bf16 *__restrict__ inb, int cb, float *__restrict__ dw,
                                                     float *__restrict__ dbias, int D, int H, int W, long long V,
                                                     int chunk) {
    __shared__ bf16 sd[BW_KV][64 + 8];       // dout rows (64 channels of this block), padded
    __shared__ bf16 sx[BW_KV][16 * NCI + 8]; // shifted input rows
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row = lane & 15, grp = lane >> 4;
    const int tap = blockIdx.x;  // the 27 taps of one voxel chunk run side by side and share L2
    const int co_blk = blockIdx.z * 64;
    const int cin = 16 * NCI;
    const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
    const int Dc = D >> 1, Hc = H >> 1, Wc = W >> 1;
    const long long v0 = (long long)blockIdx.y * chunk;
    const long long v1 = v0 + chunk < V ? v0 + chunk : V;
    f32x4 acc[NCI];
#pragma unroll
    for (int t = 0; t < NCI; t++) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    const bool wave_ok = co_blk + wave * 16 < cout;
    for (long long vb = v0; vb < v1; vb += BW_KV) {
        __syncthreads();
        // stage dout[vb .. vb+32)[co_blk .. co_blk+64) : 32 x 64 bf16, 8 per thread
        {
            const int e = threadIdx.x * 8;          // 256 threads x 8 = 2048 = 32 x 64
            const int vr = e / 64, c = e % 64;
            const long long v = vb + vr;
            bf16x8 val = zero8();
            if (v < v1 && co_blk + c < cout) val = *(const bf16x8 *)(dout + v * cout + co_blk + c);
#pragma unroll
            for (int j = 0; j < 8; j++) sd[vr][c + j] = val[j];
        }
        // stage X[v + tap shift][0 .. cin) : 32 x cin bf16, 8 per thread per pass
        for (int e = threadIdx.x * 8; e < BW_KV * cin; e += NTH * 8) {
            const int vr = e / cin, c = e % cin;
            const long long v = vb + vr;
            bf16x8 val = zero8();
            if (v < v1) {
                long long t = v;
                const int x = (int)(t % W) + dx;
                t /= W;
                const int y = (int)(t % H) + dy;
                t /= H;
                const int z = (int)(t % D) + dz;
                const int n = (int)(t / D);
                if (z >= 0 && z < D && y >= 0 && y < H && x >= 0 && x < W) {
                    if (c < ca) {
                        size_t vox;
                        if (upa) vox = (((size_t)n * Dc + (z >> 1)) * Hc + (y >> 1)) * Wc + (x >> 1);
                        else vox = (((size_t)n * D + z) * H + y) * W + x;
                        val = *(const bf16x8 *)(ina + vox * ca + c);
                    } else {
                        const size_t vox = (((size_t)n * D + z) * H + y) * W + x;
                        val = *(const bf16x8 *)(inb + vox * cb + (c - ca));
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < 8; j++) sx[vr][c + j] = val[j];
        }
        __syncthreads();
        if (wave_ok) {
            // A[m = co][k = voxel]: lane takes co = row, voxels 8*grp .. 8*grp+7
            bf16x8 afr;
#pragma unroll
            for (int j = 0; j < 8; j++) afr[j] = sd[grp * 8 + j][wave * 16 + row];
            if (tap == 13 && dbias) {
#pragma unroll
                for (int j = 0; j < 8; j++) bsum += (float)afr[j];
            }
#pragma unroll
            for (int t = 0; t < NCI; t++) {
                bf16x8 bfr;  // B[k = voxel][n = ci]
#pragma unroll
                for (int j = 0; j < 8; j++) bfr[j] = sx[grp * 8 + j][t * 16 + row];
                acc[t] = mfma(afr, bfr, acc[t]);
            }
        }
    }
    if (!wave_ok) return;
    // D[m = co][n = ci]: lane holds co = 4*grp + r, ci = row
#pragma unroll
    for (int t = 0; t < NCI; t++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int co = co_blk + wave * 16 + grp * 4 + r;
            const int ci = t * 16 + row;
            if (co < cout) atomicAdd(&dw[((size_t)tap * cout + co) * cin + ci], acc[t][r]);
        }
    if (tap == 13 && dbias) {
        // lanes with the same row hold partial sums of channel co = row over different voxel groups
        bsum += __shfl_xor(bsum, 16);
        bsum += __shfl_xor(bsum, 32);
        if (grp == 0) atomicAdd(&dbias[co_blk + wave * 16 + row], bsum);
    }
}

// ----------------------------------------------------------- elementwise
// wt[26 - tap][ci][co] = w[tap][co][ci]: the backward-data convolution is the
// forward one with flipped taps and transposed channels.
__global__ void k_flip(const bf16 *__restrict__ w, bf16 *__restrict__ wt, int cout, int cin) {
    const long long n = 27LL * cout * cin;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const int ci = (int)(e % cin);
        const int co = (int)((e / cin) % cout);
        const int tap = (int)(e / ((long long)cin * cout));
        wt[((size_t)(26 - tap) * cin + ci) * cout + co] = w[e];
    }
}

__global__ void k_relu_bwd(bf16 *__restrict__ dy, const bf16 *__restrict__ y, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        if (!((float)y[e] > 0.f)) dy[e] = (bf16)0.0f;
}

// 2x average pooling of a (N, D, H, W, C) tensor into (N, D/2, H/2, W/2, C).
__global__ void k_pool(const bf16 *__restrict__ in, bf16 *__restrict__ out, int C, int N, int D, int H, int W) {
    const int Dc = D >> 1, Hc = H >> 1, Wc = W >> 1;
    const long long n = (long long)N * Dc * Hc * Wc * C;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        long long t = e / C;
        const int x = (int)(t % Wc);
        t /= Wc;
        const int y = (int)(t % Hc);
        t /= Hc;
        const int z = (int)(t % Dc);
        const int b = (int)(t / Dc);
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const size_t vox = (((size_t)b * D + 2 * z + (q >> 2)) * H + 2 * y + ((q >> 1) & 1)) * W + 2 * x + (q & 1);
            s += (float)in[vox * C + c];
        }
        out[e] = (bf16)(0.125f * s);
    }
}

// Gradient of the pooling: din[fine] += dout[parent] / 8.
__global__ void k_pool_bwd(const bf16 *__restrict__ dout, bf16 *__restrict__ din, int C, int N, int D, int H,
                           int W) {
    const int Dc = D >> 1, Hc = H >> 1, Wc = W >> 1;
    const long long n = (long long)N * D * H * W * C;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(e % C);
        long long t = e / C;
        const int x = (int)(t % W);
        t /= W;
        const int y = (int)(t % H);
        t /= H;
        const int z = (int)(t % D);
        const int b = (int)(t / D);
        const size_t p = (((size_t)b * Dc + (z >> 1)) * Hc + (y >> 1)) * Wc + (x >> 1);
        din[e] = (bf16)((float)din[e] + 0.125f * (float)dout[p * C + c]);
    }
}

// Split the gradient of a concatenated, partly upsampled input:
// dup[coarse][c] = sum over its 8 fine children of dx[fine][c] (c < ca), and
// dskip[fine][c - ca] = dx[fine][c] (c >= ca; the pooling path adds its share later).
__global__ void k_split_grad(const bf16 *__restrict__ dx, int ca, int cb, bf16 *__restrict__ dup,
                             bf16 *__restrict__ dskip, int N, int D, int H, int W) {
    const int cin = ca + cb;
    const int Dc = D >> 1, Hc = H >> 1, Wc = W >> 1;
    const long long nc = (long long)N * Dc * Hc * Wc * ca;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nc; e += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(e % ca);
        long long t = e / ca;
        const int x = (int)(t % Wc);
        t /= Wc;
        const int y = (int)(t % Hc);
        t /= Hc;
        const int z = (int)(t % Dc);
        const int b = (int)(t / Dc);
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const size_t vox = (((size_t)b * D + 2 * z + (q >> 2)) * H + 2 * y + ((q >> 1) & 1)) * W + 2 * x + (q & 1);
            s += (float)dx[vox * cin + c];
        }
        dup[e] = (bf16)s;
    }
    if (!dskip) return;
    const long long nf = (long long)N * D * H * W * cb;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nf; e += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(e % cb);
        const long long v = e / cb;
        dskip[e] = dx[v * cin + ca + c];
    }
}

// Per-sample sums over active cells: stats[2n] = sum rho^2, stats[2n+1] =
// active count (both start at zero).
__global__ void k_stats(const double *__restrict__ rho, const int8_t *__restrict__ mask, long long vs,
                        double *__restrict__ stats) {
    __shared__ double s_a[NTH / 64], s_c[NTH / 64];
    const int n = blockIdx.y;
    double a = 0.0, c = 0.0;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < vs; v += (long long)gridDim.x * blockDim.x) {
        const long long e = n * vs + v;
        if (mask[e] == 1) {
            a += rho[e] * rho[e];
            c += 1.0;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        c += __shfl_xor(c, o);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        s_a[wv] = a;
        s_c[wv] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < NTH / 64; q++) {
            a += s_a[q];
            c += s_c[q];
        }
        atomicAdd(&stats[2 * n], a);
        atomicAdd(&stats[2 * n + 1], c);
    }
}

// Input scale of sample n: root mean square of rho over its active cells (1 if zero).
__device__ __forceinline__ double sample_scale(const double *stats, int n) {
    const double c = stats[2 * n + 1];
    const double s = c > 0.0 ? sqrt(stats[2 * n] / c) : 0.0;
    return s > 0.0 ? s : 1.0;
}

// Network input at 1/S resolution, 16 channels per voxel: mean of rho over
// the active fine cells of the block / s, +1 if more than half of the block
// is active (else -1), mean of B over the block / s, zeros.
__global__ void k_pack(const double *__restrict__ rho, const int8_t *__restrict__ mask, const double *__restrict__ B,
                       const double *__restrict__ stats, int S, int N, int Dc, int Hc, int Wc, bf16 *__restrict__ x) {
    const long long Vc = (long long)Dc * Hc * Wc;
    const long long total = (long long)N * Vc;
    const int W = Wc * S, H = Hc * S, D = Dc * S;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(e / Vc);
        long long t = e - n * Vc;
        const int cx = (int)(t % Wc);
        t /= Wc;
        const int cy = (int)(t % Hc);
        const int cz = (int)(t / Hc);
        const double is = 1.0 / sample_scale(stats, n);
        double rs = 0.0, bs = 0.0;
        int cnt = 0;
        for (int dz = 0; dz < S; dz++)
            for (int dy = 0; dy < S; dy++)
                for (int dx = 0; dx < S; dx++) {
                    const size_t f = (((size_t)n * D + cz * S + dz) * H + cy * S + dy) * W + cx * S + dx;
                    if (mask[f] == 1) {
                        rs += rho[f];
                        cnt++;
                    }
                    if (B) bs += B[f];
                }
        const int S3 = S * S * S;
        bf16x8 a = zero8(), b = zero8();
        a[0] = (bf16)(float)(cnt > 0 ? rs / cnt * is : 0.0);
        a[1] = (bf16)(2 * cnt > S3 ? 1.0f : -1.0f);
        a[2] = (bf16)(float)(bs / S3 * is);
        *(bf16x8 *)(x + e * 16) = a;
        *(bf16x8 *)(x + e * 16 + 8) = b;
    }
}

// Head: phi[v] = s_n / 256 * (sum_c w[c] x[v][c] + b), zero where a mask is
// given and the cell is inactive.
__global__ void k_head(const bf16 *__restrict__ x, const float *__restrict__ w, const float *__restrict__ b,
                       const double *__restrict__ stats, const int8_t *__restrict__ mask, double *__restrict__ phi,
                       long long vs, int N) {
    const long long V = vs * N;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
        float s = b[0];
#pragma unroll
        for (int c = 0; c < 16; c++) s += w[c] * (float)x[v * 16 + c];
        const double sc = sample_scale(stats, (int)(v / vs)) * (1.0 / 256.0);
        phi[v] = (mask == nullptr || mask[v] == 1) ? sc * (double)s : 0.0;
    }
}

// Linear up-sampling of a cell-centred field by 2 per axis: 3/4 of the
// parent plus 1/4 of the next coarse cell on the child's side (the edge cell
// repeated past the array end); zero on inactive cells when a mask is given.
__global__ void k_up2(const double *__restrict__ c, double *__restrict__ f, int N, int Dc, int Hc, int Wc,
                      const int8_t *__restrict__ mask) {
    const int D = 2 * Dc, H = 2 * Hc, W = 2 * Wc;
    const long long total = (long long)N * D * H * W;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        long long t = e;
        const int x = (int)(t % W);
        t /= W;
        const int y = (int)(t % H);
        t /= H;
        const int z = (int)(t % D);
        const int n = (int)(t / D);
        if (mask && mask[e] != 1) {
            f[e] = 0.0;
            continue;
        }
        const int px = x >> 1, py = y >> 1, pz = z >> 1;
        const int qx = min(max((x & 1) ? px + 1 : px - 1, 0), Wc - 1);
        const int qy = min(max((y & 1) ? py + 1 : py - 1, 0), Hc - 1);
        const int qz = min(max((z & 1) ? pz + 1 : pz - 1, 0), Dc - 1);
        const size_t base = (size_t)n * Dc * Hc * Wc;
        auto at = [&](int zz, int yy, int xx) { return c[base + ((size_t)zz * Hc + yy) * Wc + xx]; };
        const double z0 = 0.75 * (0.75 * at(pz, py, px) + 0.25 * at(pz, py, qx)) +
                          0.25 * (0.75 * at(pz, qy, px) + 0.25 * at(pz, qy, qx));
        const double z1 = 0.75 * (0.75 * at(qz, py, px) + 0.25 * at(qz, py, qx)) +
                          0.25 * (0.75 * at(qz, qy, px) + 0.25 * at(qz, qy, qx));
        f[e] = 0.75 * z0 + 0.25 * z1;
    }
}

// Coarse copy of a problem for a first guess: the mask keeps a block active
// when more than half of its S^3 cells are active (the outermost coarse layer
// is always inactive), rho is the mean over the active cells of the block and
// B the mean over the block.
__global__ void k_coarsen(const double *__restrict__ rho, const int8_t *__restrict__ mask, const double *__restrict__ B,
                          int S, int Dc, int Hc, int Wc, double *__restrict__ rho_c, int8_t *__restrict__ mask_c,
                          double *__restrict__ B_c) {
    const long long total = (long long)Dc * Hc * Wc;
    const int W = Wc * S, H = Hc * S;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
        long long t = e;
        const int cx = (int)(t % Wc);
        t /= Wc;
        const int cy = (int)(t % Hc);
        const int cz = (int)(t / Hc);
        double rs = 0.0, bs = 0.0;
        int cnt = 0;
        for (int dz = 0; dz < S; dz++)
            for (int dy = 0; dy < S; dy++)
                for (int dx = 0; dx < S; dx++) {
                    const size_t f = ((size_t)(cz * S + dz) * H + cy * S + dy) * W + cx * S + dx;
                    if (mask[f] == 1) {
                        rs += rho[f];
                        cnt++;
                    }
                    if (B) bs += B[f];
                }
        const int S3 = S * S * S;
        const bool frame = cx == 0 || cy == 0 || cz == 0 || cx == Wc - 1 || cy == Hc - 1 || cz == Dc - 1;
        mask_c[e] = (!frame && 2 * cnt > S3) ? 1 : -1;
        rho_c[e] = cnt > 0 ? rs / cnt : 0.0;
        if (B_c) B_c[e] = bs / S3;
    }
}

// Loss = mean over the active cells of the batch of (y - t)^2, with y the
// head output and t = 256 target / s_n.  Writes dx (bf16), accumulates the
// head's weight and bias gradients and the loss.
__global__ void k_head_loss(const bf16 *__restrict__ x, const float *__restrict__ w, const float *__restrict__ b,
                            const int8_t *__restrict__ mask, const double *__restrict__ target,
                            const double *__restrict__ stats, int N, long long vs, bf16 *__restrict__ dx,
                            float *__restrict__ dw, float *__restrict__ db, double *__restrict__ loss) {
    __shared__ float s_dw[NTH / 64][17];
    __shared__ double s_l[NTH / 64];
    double count = 0.0;
    for (int n = 0; n < N; n++) count += stats[2 * n + 1];
    const double inv_count = count > 0.0 ? 1.0 / count : 0.0;
    float ldw[17];
#pragma unroll
    for (int c = 0; c < 17; c++) ldw[c] = 0.f;
    double lsum = 0.0;
    const long long V = vs * N;
    for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V; v += (long long)gridDim.x * blockDim.x) {
        float xv[16];
        float y = b[0];
#pragma unroll
        for (int c = 0; c < 16; c++) {
            xv[c] = (float)x[v * 16 + c];
            y += w[c] * xv[c];
        }
        float g = 0.f;
        if (mask[v] == 1) {
            const double t = target[v] * 256.0 / sample_scale(stats, (int)(v / vs));
            const double d = (double)y - t;
            lsum += d * d;
            g = (float)(2.0 * d * inv_count);
        }
        bf16x8 lo, hi;
#pragma unroll
        for (int c = 0; c < 8; c++) {
            lo[c] = (bf16)(g * w[c]);
            hi[c] = (bf16)(g * w[c + 8]);
        }
        *(bf16x8 *)(dx + v * 16) = lo;
        *(bf16x8 *)(dx + v * 16 + 8) = hi;
#pragma unroll
        for (int c = 0; c < 16; c++) ldw[c] += g * xv[c];
        ldw[16] += g;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 17; c++) {
        float t = ldw[c];
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
        if (lane == 0) s_dw[wv][c] = t;
    }
    double lt = lsum;
    for (int o = 32; o > 0; o >>= 1) lt += __shfl_xor(lt, o);
    if (lane == 0) s_l[wv] = lt;
    __syncthreads();
    if (threadIdx.x < 17) {
        float t = 0.f;
        for (int q = 0; q < NTH / 64; q++) t += s_dw[q][threadIdx.x];
        if (threadIdx.x < 16) atomicAdd(&dw[threadIdx.x], t);
        else atomicAdd(db, t);
    }
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < NTH / 64; q++) t += s_l[q];
        atomicAdd(loss, t * inv_count);
    }
}

__global__ void k_fill_f32(float *__restrict__ p, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        p[e] = 0.f;
}

__global__ void k_fill_f64(double *__restrict__ p, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        p[e] = 0.0;
}

// AdamW on FP32 master weights, refreshing the BF16 copy (decoupled decay).
__global__ void k_adamw(float *__restrict__ p, bf16 *__restrict__ pb, const float *__restrict__ g, float *__restrict__ m,
                        float *__restrict__ v, long long n, float lr, float b1, float b2, float eps, float wd,
                        float c1, float c2) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const float gg = g[e];
        const float mm = b1 * m[e] + (1.f - b1) * gg;
        const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
        m[e] = mm;
        v[e] = vv;
        float w = p[e] * (1.f - lr * wd);
        w -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
        p[e] = w;
        if (pb) pb[e] = (bf16)w;
    }
}

// 16 x 16 x 32 self-test of the operand and result lane layouts with small
// integers (exact in BF16 and FP32): a[m][k] = (3m + k) mod 7 - 3,
// b[k][n] = (5k + 2n) mod 9 - 4, out[m][n] = sum_k a[m][k] b[k][n].
__global__ void k_mfma_selftest(float *out) {
    const int lane = threadIdx.x, row = lane & 15, grp = lane >> 4;
    bf16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const int k = grp * 8 + j;
        a[j] = (bf16)(float)((3 * row + k) % 7 - 3);
        b[j] = (bf16)(float)((5 * k + 2 * row) % 9 - 4);
    }
    f32x4 c = f32x4{0.f, 0.f, 0.f, 0.f};
    c = mfma(a, b, c);
#pragma unroll
    for (int r = 0; r < 4; r++) out[(grp * 4 + r) * 16 + row] = c[r];
}

inline unsigned blocks_for(long long n, int per = 256) {
    long long g = (n + per - 1) / per;
    if (g > 16384) g = 16384;
    return (unsigned)(g > 0 ? g : 1);
}

template <int NCI>
void launch_bww(const bf16 *dout, int cout, const bf16 *ina, int ca, int upa, const bf16 *inb, int cb, float *dw,
                float *db, int D, int H, int W, long long V, hipStream_t s) {
    // voxel chunk per block: about 2048 blocks over the 27 taps x channel groups
    const int groups = (cout + 63) / 64;
    long long nchunks = 2048 / (27 * groups);
    if (nchunks < 1) nchunks = 1;
    long long chunk = (V + nchunks - 1) / nchunks;
    chunk = ((chunk + BW_KV - 1) / BW_KV) * BW_KV;
    if (chunk < BW_KV) chunk = BW_KV;
    dim3 grid(27, (unsigned)((V + chunk - 1) / chunk), (unsigned)groups);
    k_conv_bwd_w<NCI><<<grid, NTH, 0, s>>>(dout, cout, ina, ca, upa, inb, cb, dw, db, D, H, W, V, (int)chunk);
}

// ------------------------------------------------ host launchers (nn_core.h)
static bool dims_ok(int n, int d, int h, int w) { return n > 0 && d > 0 && h > 0 && w > 0; }

template <int CK, int NTC>
void launch_tile(const bf16 *ina, int ca, int upa, const bf16 *inb, int cb, const bf16 *w, const float *bias, bf16 *out,
                 int cout, int relu, int n, int D, int H, int W, hipStream_t s) {
    const int ntx = (W + TX - 1) / TX, nty = (H + TY - 1) / TY, ntz = (D + TZ - 1) / TZ;
    const int nblk = n * ntx * nty * ntz;
    dim3 grid((unsigned)nblk, (unsigned)(cout / (16 * NTC)));
    if constexpr (CK == 32) {
        if ((ca + cb) % 32 == 16) {
            k_conv_tile<CK, NTC, true><<<grid, NTH, 0, s>>>(ina, ca, upa, inb, cb, w, bias, out, cout, relu, D, H, W,
                                                            ntx, nty, ntz, nblk);
            return;
        }
    }
    k_conv_tile<CK, NTC><<<grid, NTH, 0, s>>>(ina, ca, upa, inb, cb, w, bias, out, cout, relu, D, H, W, ntx, nty, ntz,
                                              nblk);
}

template <int CK>
void launch_tile_ck(const bf16 *ina, int ca, int upa, const bf16 *inb, int cb, const bf16 *w, const float *bias,
                    bf16 *out, int cout, int relu, int n, int D, int H, int W, hipStream_t s) {
    // widest output tiling that still gives about 1024 blocks
    const long long nblk = (long long)n * ((W + TX - 1) / TX) * ((H + TY - 1) / TY) * ((D + TZ - 1) / TZ);
    const int tiles = cout / 16;
    int ntc = tiles % 4 == 0 ? 4 : tiles % 2 == 0 ? 2 : 1;
    while (ntc > 1 && nblk * (tiles / ntc) < 1024) ntc /= 2;
    if (ntc == 4) launch_tile<CK, 4>(ina, ca, upa, inb, cb, w, bias, out, cout, relu, n, D, H, W, s);
    else if (ntc == 2) launch_tile<CK, 2>(ina, ca, upa, inb, cb, w, bias, out, cout, relu, n, D, H, W, s);
    else launch_tile<CK, 1>(ina, ca, upa, inb, cb, w, bias, out, cout, relu, n, D, H, W, s);
}

bool conv_fwd(const void *in_a, int ca, int up_a, const void *in_b, int cb, const void *w, const float *bias,
              void *out, int cout, int relu, int n, int d, int h, int wd, hipStream_t s) {
    if (!in_a || !w || !out || ca <= 0 || cb < 0 || (cb > 0 && !in_b) || ca % 8 || cb % 8 || cout <= 0 ||
        cout % 16 || !dims_ok(n, d, h, wd) || (up_a && (d % 2 || h % 2 || wd % 2))) {
        set_error("conv3d: invalid arguments (input channels multiples of 8, output channels of 16)");
        return false;
    }
    const bf16 *A = (const bf16 *)in_a, *B = (const bf16 *)in_b, *W = (const bf16 *)w;
    bf16 *O = (bf16 *)out;
    if (ca + cb <= 16) launch_tile_ck<16>(A, ca, up_a, B, cb, W, bias, O, cout, relu, n, d, h, wd, s);
    else launch_tile_ck<32>(A, ca, up_a, B, cb, W, bias, O, cout, relu, n, d, h, wd, s);
    return hip_ok(hipGetLastError(), "conv3d launch");
}

bool conv_bwd_weight(const void *dout, int cout, const void *in_a, int ca, int up_a, const void *in_b, int cb,
                     float *dw, float *dbias, int n, int d, int h, int wd, hipStream_t s) {
    const int cin = ca + cb;
    if (!dout || !in_a || !dw || cout <= 0 || cout % 16 || ca <= 0 || ca % 8 || cb < 0 || cb % 8 ||
        (cb > 0 && !in_b) || cin % 16 || !dims_ok(n, d, h, wd) || (up_a && (d % 2 || h % 2 || wd % 2))) {
        set_error("conv3d weight gradient: invalid arguments (input channels a multiple of 16, output of 16)");
        return false;
    }
    const long long V = (long long)n * d * h * wd;
    const bf16 *G = (const bf16 *)dout, *A = (const bf16 *)in_a, *B = (const bf16 *)in_b;
    switch (cin / 16) {
        case 1: launch_bww<1>(G, cout, A, ca, up_a, B, cb, dw, dbias, d, h, wd, V, s); break;
        case 2: launch_bww<2>(G, cout, A, ca, up_a, B, cb, dw, dbias, d, h, wd, V, s); break;
        case 3: launch_bww<3>(G, cout, A, ca, up_a, B, cb, dw, dbias, d, h, wd, V, s); break;
        case 4: launch_bww<4>(G, cout, A, ca, up_a, B, cb, dw, dbias, d, h, wd, V, s); break;
        case 6: launch_bww<6>(G, cout, A, ca, up_a, B, cb, dw, dbias, d, h, wd, V, s); break;
        case 8: launch_bww<8>(G, cout, A, ca, up_a, B, cb, dw, dbias, d, h, wd, V, s); break;
        case 12: launch_bww<12>(G, cout, A, ca, up_a, B, cb, dw, dbias, d, h, wd, V, s); break;
        default:
            set_error("conv3d weight gradient: input channels must be 16, 32, 48, 64, 96, 128 or 192");
            return false;
    }
    return hip_ok(hipGetLastError(), "conv3d weight gradient launch");
}

bool weight_flip(const void *w, int cout, int cin, void *wt, hipStream_t s) {
    const long long n = 27LL * cout * cin;
    k_flip<<<blocks_for(n), 256, 0, s>>>((const bf16 *)w, (bf16 *)wt, cout, cin);
    return hip_ok(hipGetLastError(), "weight flip launch");
}

bool relu_bwd(void *dy, const void *y, long long count, hipStream_t s) {
    k_relu_bwd<<<blocks_for(count), 256, 0, s>>>((bf16 *)dy, (const bf16 *)y, count);
    return hip_ok(hipGetLastError(), "relu backward launch");
}

bool pool2(const void *in, void *out, int c, int n, int d, int h, int wd, hipStream_t s) {
    const long long cnt = (long long)n * (d / 2) * (h / 2) * (wd / 2) * c;
    k_pool<<<blocks_for(cnt), 256, 0, s>>>((const bf16 *)in, (bf16 *)out, c, n, d, h, wd);
    return hip_ok(hipGetLastError(), "pool launch");
}

bool pool2_bwd(const void *dout, void *din, int c, int n, int d, int h, int wd, hipStream_t s) {
    const long long cnt = (long long)n * d * h * wd * c;
    k_pool_bwd<<<blocks_for(cnt), 256, 0, s>>>((const bf16 *)dout, (bf16 *)din, c, n, d, h, wd);
    return hip_ok(hipGetLastError(), "pool backward launch");
}

bool split_grad(const void *dx, int ca, int cb, void *dup, void *dskip, int n, int d, int h, int wd, hipStream_t s) {
    const long long cnt = (long long)n * d * h * wd * (ca > cb ? ca : cb);
    k_split_grad<<<blocks_for(cnt), 256, 0, s>>>((const bf16 *)dx, ca, cb, (bf16 *)dup, (bf16 *)dskip, n, d, h, wd);
    return hip_ok(hipGetLastError(), "split gradient launch");
}

bool stats(const double *rho, const int8_t *mask, long long vs, int n, double *st, hipStream_t s) {
    k_fill_f64<<<1, 64, 0, s>>>(st, 2LL * n);
    dim3 grid(blocks_for(vs, 4096), (unsigned)n);
    k_stats<<<grid, NTH, 0, s>>>(rho, mask, vs, st);
    return hip_ok(hipGetLastError(), "stats launch");
}

bool pack(const double *rho, const int8_t *mask, const double *B, const double *st, int S, int n, int dc, int hc,
          int wc, void *x, hipStream_t s) {
    const long long total = (long long)n * dc * hc * wc;
    k_pack<<<blocks_for(total), 256, 0, s>>>(rho, mask, B, st, S, n, dc, hc, wc, (bf16 *)x);
    return hip_ok(hipGetLastError(), "pack launch");
}

bool head(const void *x, const float *w, const float *b, const double *st, const int8_t *mask, double *phi,
          long long vs, int n, hipStream_t s) {
    k_head<<<blocks_for(vs * n), 256, 0, s>>>((const bf16 *)x, w, b, st, mask, phi, vs, n);
    return hip_ok(hipGetLastError(), "head launch");
}

bool up2(const double *c, double *f, int n, int dc, int hc, int wc, const int8_t *mask, hipStream_t s) {
    k_up2<<<blocks_for(8LL * n * dc * hc * wc), 256, 0, s>>>(c, f, n, dc, hc, wc, mask);
    return hip_ok(hipGetLastError(), "up-sampling launch");
}

bool coarsen(const double *rho, const int8_t *mask, const double *B, int S, int dc, int hc, int wc, double *rho_c,
             int8_t *mask_c, double *B_c, hipStream_t s) {
    k_coarsen<<<blocks_for((long long)dc * hc * wc), 256, 0, s>>>(rho, mask, B, S, dc, hc, wc, rho_c, mask_c, B_c);
    return hip_ok(hipGetLastError(), "coarsen launch");
}

bool head_loss(const void *x, const float *w, const float *b, const int8_t *mask, const double *target,
               const double *st, int n, long long vs, void *dx, float *dw, float *db, double *loss, hipStream_t s) {
    k_head_loss<<<blocks_for(vs * n, 1024), NTH, 0, s>>>((const bf16 *)x, w, b, mask, target, st, n, vs, (bf16 *)dx,
                                                         dw, db, loss);
    return hip_ok(hipGetLastError(), "loss launch");
}

bool fill_f32(float *p, long long n, hipStream_t s) {
    k_fill_f32<<<blocks_for(n), 256, 0, s>>>(p, n);
    return hip_ok(hipGetLastError(), "fill launch");
}

bool fill_f64(double *p, long long n, hipStream_t s) {
    k_fill_f64<<<blocks_for(n), 256, 0, s>>>(p, n);
    return hip_ok(hipGetLastError(), "fill launch");
}

bool adamw(float *p, void *pb, const float *g, float *m, float *v, long long n, float lr, float b1, float b2, float eps,
           float wd, int step, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    k_adamw<<<blocks_for(n), 256, 0, s>>>(p, (bf16 *)pb, g, m, v, n, lr, b1, b2, eps, wd, c1, c2);
    return hip_ok(hipGetLastError(), "adamw launch");
}

}  // namespace nn
}  // namespace mg

using namespace mg;

#define NN_RET(x) return (x) ? MG_OK : MG_ERR_HIP

extern "C" {

mg_status mg_nn_conv3d_fwd(const void *in_a, int32_t ca, int32_t up_a, const void *in_b, int32_t cb, const void *w,
                           const float *bias, void *out, int32_t cout, int32_t relu, int32_t n, int32_t d, int32_t h,
                           int32_t wd, void *stream) {
    if (!in_a || !w || !out || ca <= 0 || cb < 0 || (cb > 0 && !in_b) || ca % 8 || cb % 8 || cout <= 0 || cout % 16 ||
        n <= 0 || d <= 0 || h <= 0 || wd <= 0 || (up_a && (d % 2 || h % 2 || wd % 2))) {
        set_error("mg_nn_conv3d_fwd: invalid arguments");
        return MG_ERR_ARG;
    }
    NN_RET(nn::conv_fwd(in_a, ca, up_a, in_b, cb, w, bias, out, cout, relu, n, d, h, wd, (hipStream_t)stream));
}

mg_status mg_nn_conv3d_bwd_weight(const void *dout, int32_t cout, const void *in_a, int32_t ca, int32_t up_a,
                                  const void *in_b, int32_t cb, float *dw, float *dbias, int32_t n, int32_t d,
                                  int32_t h, int32_t wd, void *stream) {
    const int cin = ca + cb;
    const bool cin_ok = cin == 16 || cin == 32 || cin == 48 || cin == 64 || cin == 96 || cin == 128 || cin == 192;
    if (!dout || !in_a || !dw || cout <= 0 || cout % 16 || ca <= 0 || ca % 8 || cb < 0 || cb % 8 ||
        (cb > 0 && !in_b) || !cin_ok || n <= 0 || d <= 0 || h <= 0 || wd <= 0 ||
        (up_a && (d % 2 || h % 2 || wd % 2))) {
        set_error("mg_nn_conv3d_bwd_weight: invalid arguments");
        return MG_ERR_ARG;
    }
    NN_RET(nn::conv_bwd_weight(dout, cout, in_a, ca, up_a, in_b, cb, dw, dbias, n, d, h, wd, (hipStream_t)stream));
}

mg_status mg_nn_weight_flip(const void *w, int32_t cout, int32_t cin, void *wt, void *stream) {
    if (!w || !wt || cout <= 0 || cin <= 0) {
        set_error("mg_nn_weight_flip: invalid arguments");
        return MG_ERR_ARG;
    }
    NN_RET(nn::weight_flip(w, cout, cin, wt, (hipStream_t)stream));
}

mg_status mg_nn_relu_bwd(void *dy, const void *y, int64_t count, void *stream) {
    if (!dy || !y || count <= 0) {
        set_error("mg_nn_relu_bwd: invalid arguments");
        return MG_ERR_ARG;
    }
    NN_RET(nn::relu_bwd(dy, y, count, (hipStream_t)stream));
}

mg_status mg_nn_pool2(const void *in, void *out, int32_t c, int32_t n, int32_t d, int32_t h, int32_t wd, void *stream) {
    if (!in || !out || c <= 0 || n <= 0 || d <= 0 || h <= 0 || wd <= 0 || d % 2 || h % 2 || wd % 2) {
        set_error("mg_nn_pool2: invalid arguments");
        return MG_ERR_ARG;
    }
    NN_RET(nn::pool2(in, out, c, n, d, h, wd, (hipStream_t)stream));
}

mg_status mg_nn_pool2_bwd(const void *dout, void *din, int32_t c, int32_t n, int32_t d, int32_t h, int32_t wd,
                          void *stream) {
    if (!dout || !din || c <= 0 || n <= 0 || d <= 0 || h <= 0 || wd <= 0 || d % 2 || h % 2 || wd % 2) {
        set_error("mg_nn_pool2_bwd: invalid arguments");
        return MG_ERR_ARG;
    }
    NN_RET(nn::pool2_bwd(dout, din, c, n, d, h, wd, (hipStream_t)stream));
}

mg_status mg_nn_split_grad(const void *dx, int32_t ca, int32_t cb, void *dup, void *dskip, int32_t n, int32_t d,
                           int32_t h, int32_t wd, void *stream) {
    if (!dx || !dup || ca <= 0 || cb < 0 || (cb > 0 && !dskip) || n <= 0 || d <= 0 || h <= 0 || wd <= 0 || d % 2 ||
        h % 2 || wd % 2) {
        set_error("mg_nn_split_grad: invalid arguments");
        return MG_ERR_ARG;
    }
    NN_RET(nn::split_grad(dx, ca, cb, dup, dskip, n, d, h, wd, (hipStream_t)stream));
}

mg_status mg_nn_adamw(float *param, void *param_bf16, const float *grad, float *m, float *v, int64_t count, float lr,
                      float beta1, float beta2, float eps, float weight_decay, int32_t step, void *stream) {
    if (!param || !grad || !m || !v || count <= 0 || step < 1) {
        set_error("mg_nn_adamw: invalid arguments");
        return MG_ERR_ARG;
    }
    NN_RET(nn::adamw(param, param_bf16, grad, m, v, count, lr, beta1, beta2, eps, weight_decay, step,
                     (hipStream_t)stream));
}

mg_status mg_nn_mfma_selftest(float *out_dev, void *stream) {
    if (!out_dev) {
        set_error("mg_nn_mfma_selftest: null output");
        return MG_ERR_ARG;
    }
    nn::k_mfma_selftest<<<1, 64, 0, (hipStream_t)stream>>>(out_dev);
    return hip_ok(hipGetLastError(), "mfma selftest launch") ? MG_OK : MG_ERR_HIP;
}

}  // extern "C"
