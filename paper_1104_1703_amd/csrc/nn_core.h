// Host launchers of the U-Net kernels (nn.hip), used by the network runtime
// (unet.hip).  Tensors are BF16 channels-last unless noted; each launcher
// enqueues on stream s and returns false after recording an error message.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mg {
namespace nn {

// out = [ReLU](conv3x3x3(concat(up2?(in_a), in_b)) + bias); weights [27][cout][cin].
bool conv_fwd(const void *in_a, int ca, int up_a, const void *in_b, int cb, const void *w, const float *bias,
              void *out, int cout, int relu, int n, int d, int h, int wd, hipStream_t s);
// dw[27][cout][cin] += weight gradient, dbias[cout] += bias gradient (FP32, atomics).
bool conv_bwd_weight(const void *dout, int cout, const void *in_a, int ca, int up_a, const void *in_b, int cb,
                     float *dw, float *dbias, int n, int d, int h, int wd, hipStream_t s);
// wt[26 - tap][ci][co] = w[tap][co][ci]
bool weight_flip(const void *w, int cout, int cin, void *wt, hipStream_t s);
bool relu_bwd(void *dy, const void *y, long long count, hipStream_t s);
bool pool2(const void *in, void *out, int c, int n, int d, int h, int wd, hipStream_t s);
bool pool2_bwd(const void *dout, void *din, int c, int n, int d, int h, int wd, hipStream_t s);
bool split_grad(const void *dx, int ca, int cb, void *dup, void *dskip, int n, int d, int h, int wd, hipStream_t s);
// st[2n] = sum of rho^2 over active cells of sample n, st[2n+1] = their count (FP64)
bool stats(const double *rho, const int8_t *mask, long long vs, int n, double *st, hipStream_t s);
bool pack(const double *rho, const int8_t *mask, const double *B, const double *st, int S, int n, int dc, int hc,
          int wc, void *x, hipStream_t s);
bool head(const void *x, const float *w, const float *b, const double *st, const int8_t *mask, double *phi,
          long long vs, int n, hipStream_t s);
bool up2(const double *c, double *f, int n, int dc, int hc, int wc, const int8_t *mask, hipStream_t s);
bool coarsen(const double *rho, const int8_t *mask, const double *B, int S, int dc, int hc, int wc, double *rho_c,
             int8_t *mask_c, double *B_c, hipStream_t s);
bool head_loss(const void *x, const float *w, const float *b, const int8_t *mask, const double *target,
               const double *st, int n, long long vs, void *dx, float *dw, float *db, double *loss, hipStream_t s);
bool fill_f32(float *p, long long n, hipStream_t s);
bool fill_f64(double *p, long long n, hipStream_t s);
bool adamw(float *p, void *pb, const float *g, float *m, float *v, long long n, float lr, float b1, float b2, float eps,
           float wd, int step, hipStream_t s);

}  // namespace nn
}  // namespace mg
