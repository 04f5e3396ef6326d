// Runtime of the learned initial guess: a 3D U-Net (4 resolutions with 16,
// 32, 64 and 128 channels, two 3x3x3 convolutions + ReLU per stage, 2x mean
// pooling, nearest up-sampling with concatenated skips, 1x1x1 head) trained
// and evaluated entirely in this library's kernels (nn.hip).
//
// The multigrid method converges from any first guess (Sec. 2); the network
// only replaces the zero start, and the FP64 stopping test of the V-cycle
// iteration (Sec. 6) is unchanged.  Conventions of the network (the input
// channels and their scale, the parameter layout) are stated in mg.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "mg.h"
#include "mg_core.h"
#include "nn_core.h"

using mg::hip_ok;
using mg::set_error;

namespace {

typedef __bf16 bf16;

enum { E1A, E1B, E2A, E2B, E3A, E3B, M4A, M4B, D3A, D3B, D2A, D2B, D1A, D1B, NLAYER };

struct LayerDef {
    int ca;     // channels of the up-sampled (half-resolution) input
    int cb;     // channels of the full-resolution input
    int cout;
    int level;  // 1 = input resolution
};

const LayerDef kLayers[NLAYER] = {
    {0, 16, 16, 1},   {0, 16, 16, 1},  {0, 16, 32, 2},  {0, 32, 32, 2}, {0, 32, 64, 3},
    {0, 64, 64, 3},   {0, 64, 128, 4}, {0, 128, 128, 4}, {128, 64, 64, 3}, {0, 64, 64, 3},
    {64, 32, 32, 2},  {0, 32, 32, 2},  {32, 16, 16, 1}, {0, 16, 16, 1},
};

__global__ void k_to_bf16(const float *__restrict__ p, bf16 *__restrict__ q, long long n) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        q[e] = (bf16)p[e];
}

// splitmix64 (Steele, Lea and Flood 2014) and the Box-Muller transform for
// the initial weights
struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal() { return sqrt(-2.0 * log(uniform())) * cos(6.283185307179586 * uniform()); }
};

}  // namespace

struct mg_unet {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    mg_allocator alloc{};
    long long np = 0;
    long long woff[NLAYER], boff[NLAYER], head_w = 0, head_b = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    bf16 *pb = nullptr, *pf = nullptr;  // BF16 weights and their flipped copies (same offsets)
    int step = 0;
    double *st = nullptr;  // per-sample input statistics
    int st_cap = 0;
    double *loss_dev = nullptr, *loss_host = nullptr;
    std::vector<void *> fixed;  // parameter-sized buffers

    // workspace of the current shape
    int wn = 0, wd = 0, wh = 0, ww = 0;
    bool wtrain = false;
    std::vector<void *> ws;
    void *x0 = nullptr, *act[NLAYER] = {}, *pool[3] = {};
    void *gact[NLAYER] = {}, *gpool[3] = {}, *gcat = nullptr;
    double *yc = nullptr, *up_tmp[2] = {};
    long long yc_len = 0, up_len[2] = {0, 0};
};

namespace {

void *raw_alloc(mg_unet *U, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (U->alloc.alloc) p = U->alloc.alloc(bytes, U->alloc.ctx);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (!p) set_error("device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
}

void raw_free(mg_unet *U, void *p) {
    if (!p) return;
    if (U->alloc.alloc) {
        if (U->alloc.free) U->alloc.free(p, U->alloc.ctx);
    } else {
        (void)hipFree(p);
    }
}

void free_workspace(mg_unet *U) {
    if (!U->ws.empty()) (void)hipStreamSynchronize(U->stream);
    for (void *p : U->ws) raw_free(U, p);
    U->ws.clear();
    U->x0 = U->gcat = nullptr;
    for (int l = 0; l < NLAYER; l++) U->act[l] = U->gact[l] = nullptr;
    for (int i = 0; i < 3; i++) U->pool[i] = U->gpool[i] = nullptr;
    U->wn = U->wd = U->wh = U->ww = 0;
    U->wtrain = false;
}

// Activations (and, for training, their gradients) for n samples of d x h x w.
bool ensure_workspace(mg_unet *U, int n, int d, int h, int w, bool train) {
    if (U->wn == n && U->wd == d && U->wh == h && U->ww == w && (U->wtrain || !train)) return true;
    free_workspace(U);
    const long long V1 = (long long)n * d * h * w;
    auto vox = [&](int level) { return V1 >> (3 * (level - 1)); };
    auto get = [&](long long elems) -> void * {
        void *p = raw_alloc(U, (size_t)elems * sizeof(bf16));
        if (p) U->ws.push_back(p);
        return p;
    };
    bool ok = true;
    ok &= (U->x0 = get(16 * V1)) != nullptr;
    for (int l = 0; l < NLAYER; l++) ok &= (U->act[l] = get(kLayers[l].cout * vox(kLayers[l].level))) != nullptr;
    ok &= (U->pool[0] = get(16 * vox(2))) != nullptr;
    ok &= (U->pool[1] = get(32 * vox(3))) != nullptr;
    ok &= (U->pool[2] = get(64 * vox(4))) != nullptr;
    if (ok && train) {
        for (int l = 0; l < NLAYER; l++)
            ok &= (U->gact[l] = get(kLayers[l].cout * vox(kLayers[l].level))) != nullptr;
        ok &= (U->gpool[0] = get(16 * vox(2))) != nullptr;
        ok &= (U->gpool[1] = get(32 * vox(3))) != nullptr;
        ok &= (U->gpool[2] = get(64 * vox(4))) != nullptr;
        long long cat = 48 * vox(1);
        if (96 * vox(2) > cat) cat = 96 * vox(2);
        if (192 * vox(3) > cat) cat = 192 * vox(3);
        ok &= (U->gcat = get(cat)) != nullptr;
    }
    if (!ok) {
        free_workspace(U);
        return false;
    }
    U->wn = n, U->wd = d, U->wh = h, U->ww = w, U->wtrain = train;
    return true;
}

bool ensure_stats(mg_unet *U, int n) {
    if (n <= U->st_cap) return true;
    if (U->st) {
        (void)hipStreamSynchronize(U->stream);
        raw_free(U, U->st);
    }
    U->st = (double *)raw_alloc(U, 2 * sizeof(double) * n);
    U->st_cap = U->st ? n : 0;
    return U->st != nullptr;
}

// Grow-only FP64 buffer for the network output and its up-sampling steps.
bool ensure_f64(mg_unet *U, double *&buf, long long &len, long long need) {
    if (need <= len) return true;
    if (buf) {
        (void)hipStreamSynchronize(U->stream);
        raw_free(U, buf);
    }
    buf = (double *)raw_alloc(U, need * sizeof(double));
    len = buf ? need : 0;
    return buf != nullptr;
}

bool refresh_weights(mg_unet *U) {
    k_to_bf16<<<2048, 256, 0, U->stream>>>(U->p, U->pb, U->np);
    if (!hip_ok(hipGetLastError(), "weight conversion launch")) return false;
    for (int l = 0; l < NLAYER; l++) {
        const int cin = kLayers[l].ca + kLayers[l].cb;
        if (!mg::nn::weight_flip(U->pb + U->woff[l], kLayers[l].cout, cin, U->pf + U->woff[l], U->stream))
            return false;
    }
    return true;
}

// Forward pass over the workspace; x0 holds the packed input.
bool forward(mg_unet *U) {
    const int n = U->wn;
    auto conv = [&](int l, const void *a, int ca, int up, const void *b, int cb) {
        const int lv = kLayers[l].level - 1;
        return mg::nn::conv_fwd(a, ca, up, b, cb, U->pb + U->woff[l], U->p + U->boff[l], U->act[l], kLayers[l].cout,
                                1, n, U->wd >> lv, U->wh >> lv, U->ww >> lv, U->stream);
    };
    auto pool = [&](const void *in, void *out, int c, int level) {
        const int lv = level - 1;
        return mg::nn::pool2(in, out, c, n, U->wd >> lv, U->wh >> lv, U->ww >> lv, U->stream);
    };
    void **A = U->act;
    return conv(E1A, U->x0, 16, 0, nullptr, 0) && conv(E1B, A[E1A], 16, 0, nullptr, 0) &&
           pool(A[E1B], U->pool[0], 16, 1) && conv(E2A, U->pool[0], 16, 0, nullptr, 0) &&
           conv(E2B, A[E2A], 32, 0, nullptr, 0) && pool(A[E2B], U->pool[1], 32, 2) &&
           conv(E3A, U->pool[1], 32, 0, nullptr, 0) && conv(E3B, A[E3A], 64, 0, nullptr, 0) &&
           pool(A[E3B], U->pool[2], 64, 3) && conv(M4A, U->pool[2], 64, 0, nullptr, 0) &&
           conv(M4B, A[M4A], 128, 0, nullptr, 0) && conv(D3A, A[M4B], 128, 1, A[E3B], 64) &&
           conv(D3B, A[D3A], 64, 0, nullptr, 0) && conv(D2A, A[D3B], 64, 1, A[E2B], 32) &&
           conv(D2B, A[D2A], 32, 0, nullptr, 0) && conv(D1A, A[D2B], 32, 1, A[E1B], 16) &&
           conv(D1B, A[D1A], 16, 0, nullptr, 0);
}

// Backward pass: gact[D1B] holds the loss gradient of the last activation.
// Weight gradients accumulate into g (cleared by the caller).
bool backward(mg_unet *U) {
    const int n = U->wn;
    hipStream_t s = U->stream;
    auto dims = [&](int level, int &d, int &h, int &w) {
        d = U->wd >> (level - 1), h = U->wh >> (level - 1), w = U->ww >> (level - 1);
    };
    // ReLU backward, weight and bias gradients, and (if dx) the gradient of
    // the layer's (concatenated) input written to dx.
    auto back = [&](int l, const void *a, int up, const void *b, void *dx) {
        const LayerDef &L = kLayers[l];
        int d, h, w;
        dims(L.level, d, h, w);
        const long long cnt = (long long)n * d * h * w * L.cout;
        const int ca = up ? L.ca : L.cb, cb = up ? L.cb : 0;
        if (!mg::nn::relu_bwd(U->gact[l], U->act[l], cnt, s)) return false;
        if (!mg::nn::conv_bwd_weight(U->gact[l], L.cout, a, ca, up, b, cb, U->g + U->woff[l], U->g + U->boff[l], n, d,
                                     h, w, s))
            return false;
        if (!dx) return true;
        return mg::nn::conv_fwd(U->gact[l], L.cout, 0, nullptr, 0, U->pf + U->woff[l], nullptr, dx, L.ca + L.cb, 0, n,
                                d, h, w, s);
    };
    auto split = [&](int level, int ca, int cb, void *dup, void *dskip) {
        int d, h, w;
        dims(level, d, h, w);
        return mg::nn::split_grad(U->gcat, ca, cb, dup, dskip, n, d, h, w, s);
    };
    auto pool_back = [&](void *gp, void *gfine, int c, int level) {
        int d, h, w;
        dims(level, d, h, w);
        return mg::nn::pool2_bwd(gp, gfine, c, n, d, h, w, s);
    };
    void **A = U->act, **G = U->gact;
    return back(D1B, A[D1A], 0, nullptr, G[D1A]) && back(D1A, A[D2B], 1, A[E1B], U->gcat) &&
           split(1, 32, 16, G[D2B], G[E1B]) && back(D2B, A[D2A], 0, nullptr, G[D2A]) &&
           back(D2A, A[D3B], 1, A[E2B], U->gcat) && split(2, 64, 32, G[D3B], G[E2B]) &&
           back(D3B, A[D3A], 0, nullptr, G[D3A]) && back(D3A, A[M4B], 1, A[E3B], U->gcat) &&
           split(3, 128, 64, G[M4B], G[E3B]) && back(M4B, A[M4A], 0, nullptr, G[M4A]) &&
           back(M4A, U->pool[2], 0, nullptr, U->gpool[2]) && pool_back(U->gpool[2], G[E3B], 64, 3) &&
           back(E3B, A[E3A], 0, nullptr, G[E3A]) && back(E3A, U->pool[1], 0, nullptr, U->gpool[1]) &&
           pool_back(U->gpool[1], G[E2B], 32, 2) && back(E2B, A[E2A], 0, nullptr, G[E2A]) &&
           back(E2A, U->pool[0], 0, nullptr, U->gpool[0]) && pool_back(U->gpool[0], G[E1B], 16, 1) &&
           back(E1B, A[E1A], 0, nullptr, G[E1A]) && back(E1A, U->x0, 0, nullptr, nullptr);
}

bool shape_ok(int n, int nx, int ny, int nz, int stride) {
    if (n <= 0 || nx <= 0 || ny <= 0 || nz <= 0) return false;
    if (stride != 1 && stride != 2 && stride != 4 && stride != 8) return false;
    const int q = 8 * stride;
    return nx % q == 0 && ny % q == 0 && nz % q == 0;
}

mg_status loss_grad(mg_unet *U, int32_t n, const double *rho, const int8_t *mask, const double *dirichlet,
                    const double *target, int32_t nx, int32_t ny, int32_t nz, double *loss_out, bool sync) {
    if (!U || !rho || !mask || !target || !shape_ok(n, nx, ny, nz, 1)) {
        set_error("mg_unet_loss_grad: invalid arguments (dims must be multiples of 8)");
        return MG_ERR_ARG;
    }
    if (!ensure_workspace(U, n, nz, ny, nx, true) || !ensure_stats(U, n)) return MG_ERR_ALLOC;
    const long long vs = (long long)nx * ny * nz;
    hipStream_t s = U->stream;
    bool ok = mg::nn::stats(rho, mask, vs, n, U->st, s) &&
              mg::nn::pack(rho, mask, dirichlet, U->st, 1, n, nz, ny, nx, U->x0, s) && forward(U) &&
              mg::nn::fill_f32(U->g, U->np, s) && mg::nn::fill_f64(U->loss_dev, 1, s) &&
              mg::nn::head_loss(U->act[D1B], U->p + U->head_w, U->p + U->head_b, mask, target, U->st, n, vs,
                                U->gact[D1B], U->g + U->head_w, U->g + U->head_b, U->loss_dev, s) &&
              backward(U);
    if (!ok) return MG_ERR_HIP;
    if (sync || loss_out) {
        if (!hip_ok(hipMemcpyAsync(U->loss_host, U->loss_dev, sizeof(double), hipMemcpyDeviceToHost, s),
                    "loss readback") ||
            !hip_ok(hipStreamSynchronize(s), "loss readback sync"))
            return MG_ERR_HIP;
        if (loss_out) *loss_out = *U->loss_host;
    }
    return MG_OK;
}

// ---- safetensors (8-byte little-endian header length, JSON header, data) ----
bool find_tensor(const std::string &hdr, const std::string &name, std::string &dtype, std::vector<long long> &shape,
                 long long &o0, long long &o1) {
    const size_t k = hdr.find("\"" + name + "\"");
    if (k == std::string::npos) return false;
    const size_t b = hdr.find('{', k), e = hdr.find('}', k);
    if (b == std::string::npos || e == std::string::npos || e < b) return false;
    const std::string body = hdr.substr(b, e - b);
    size_t t = body.find("\"dtype\"");
    if (t == std::string::npos) return false;
    t = body.find('"', body.find(':', t));
    dtype = body.substr(t + 1, body.find('"', t + 1) - t - 1);
    t = body.find("\"shape\"");
    if (t == std::string::npos) return false;
    shape.clear();
    const size_t sb = body.find('[', t), se = body.find(']', t);
    std::string sh = body.substr(sb + 1, se - sb - 1);
    for (char *c = &sh[0]; *c;) {
        char *end;
        const long long v = strtoll(c, &end, 10);
        if (end == c) {
            c++;
            continue;
        }
        shape.push_back(v);
        c = end;
    }
    t = body.find("\"data_offsets\"");
    if (t == std::string::npos) return false;
    const size_t ob = body.find('[', t);
    char *end;
    o0 = strtoll(body.c_str() + ob + 1, &end, 10);
    while (*end == ' ' || *end == ',') end++;
    o1 = strtoll(end, &end, 10);
    return true;
}

}  // namespace

extern "C" {

int64_t mg_unet_num_params(const mg_unet *U) { return U ? U->np : 0; }

mg_status mg_unet_create(uint64_t seed, const mg_allocator *alloc, void *stream, mg_unet **out) {
    if (!out) {
        set_error("mg_unet_create: null output");
        return MG_ERR_ARG;
    }
    *out = nullptr;
    mg_unet *U = new (std::nothrow) mg_unet();
    if (!U) return MG_ERR_ALLOC;
    if (alloc) U->alloc = *alloc;
    if (stream) {
        U->stream = (hipStream_t)stream;
    } else {
        if (!hip_ok(hipStreamCreate(&U->stream), "hipStreamCreate")) {
            delete U;
            return MG_ERR_HIP;
        }
        U->own_stream = true;
    }
    long long off = 0;
    for (int l = 0; l < NLAYER; l++) {
        const int cin = kLayers[l].ca + kLayers[l].cb;
        U->woff[l] = off;
        U->boff[l] = off + 27LL * kLayers[l].cout * cin;
        off = U->boff[l] + kLayers[l].cout;
    }
    U->head_w = off;
    U->head_b = off + 16;
    U->np = off + 17;
    const size_t fb = U->np * sizeof(float), hb = U->np * sizeof(bf16);
    U->p = (float *)raw_alloc(U, fb);
    U->g = (float *)raw_alloc(U, fb);
    U->m = (float *)raw_alloc(U, fb);
    U->v = (float *)raw_alloc(U, fb);
    U->pb = (bf16 *)raw_alloc(U, hb);
    U->pf = (bf16 *)raw_alloc(U, hb);
    U->loss_dev = (double *)raw_alloc(U, sizeof(double));
    for (void *p : {(void *)U->p, (void *)U->g, (void *)U->m, (void *)U->v, (void *)U->pb, (void *)U->pf,
                    (void *)U->loss_dev})
        if (p) U->fixed.push_back(p);
    if (U->fixed.size() != 7 || hipHostMalloc((void **)&U->loss_host, sizeof(double)) != hipSuccess) {
        mg_unet_destroy(U);
        set_error("mg_unet_create: allocation failed");
        return MG_ERR_ALLOC;
    }
    // He-normal weights, zero biases
    std::vector<float> h(U->np, 0.f);
    Rng rng{seed};
    for (int l = 0; l < NLAYER; l++) {
        const double sd = sqrt(2.0 / (27.0 * (kLayers[l].ca + kLayers[l].cb)));
        for (long long i = U->woff[l]; i < U->boff[l]; i++) h[i] = (float)(sd * rng.normal());
    }
    for (int c = 0; c < 16; c++) h[U->head_w + c] = (float)(0.25 * rng.normal());
    const mg_status st = mg_unet_set_params(U, h.data(), U->np);
    if (st != MG_OK) {
        mg_unet_destroy(U);
        return st;
    }
    *out = U;
    return MG_OK;
}

void mg_unet_destroy(mg_unet *U) {
    if (!U) return;
    if (U->stream) (void)hipStreamSynchronize(U->stream);
    free_workspace(U);
    for (void *p : U->fixed) raw_free(U, p);
    raw_free(U, U->st);
    raw_free(U, U->yc);
    raw_free(U, U->up_tmp[0]);
    raw_free(U, U->up_tmp[1]);
    if (U->loss_host) (void)hipHostFree(U->loss_host);
    if (U->own_stream && U->stream) (void)hipStreamDestroy(U->stream);
    delete U;
}

mg_status mg_unet_tensor(mg_unet *U, int32_t kind, int32_t index, void *dst, int64_t count) {
    if (!U || !dst || U->wn == 0) {
        set_error("mg_unet_tensor: null argument or no workspace");
        return MG_ERR_ARG;
    }
    const long long V1 = (long long)U->wn * U->wd * U->wh * U->ww;
    auto vox = [&](int level) { return V1 >> (3 * (level - 1)); };
    const void *src = nullptr;
    long long n = 0;
    if ((kind == MG_UNET_ACT || kind == MG_UNET_ACT_GRAD) && index >= 0 && index < NLAYER) {
        src = kind == MG_UNET_ACT ? U->act[index] : U->gact[index];
        n = kLayers[index].cout * vox(kLayers[index].level);
    } else if ((kind == MG_UNET_POOL || kind == MG_UNET_POOL_GRAD) && index >= 0 && index < 3) {
        src = kind == MG_UNET_POOL ? U->pool[index] : U->gpool[index];
        n = (16LL << index) * vox(index + 2);
    } else if (kind == MG_UNET_INPUT && index == 0) {
        src = U->x0;
        n = 16 * V1;
    } else if (kind == MG_UNET_CAT_GRAD && index == 0) {
        src = U->gcat;
        n = (kLayers[D3A].ca + kLayers[D3A].cb) * vox(kLayers[D3A].level);
    }
    if (!src || count != n) {
        set_error("mg_unet_tensor: no such tensor or wrong element count");
        return MG_ERR_ARG;
    }
    const bool ok = hip_ok(hipMemcpyAsync(dst, src, (size_t)n * sizeof(bf16), hipMemcpyDeviceToDevice, U->stream),
                           "tensor copy") &&
                    hip_ok(hipStreamSynchronize(U->stream), "tensor copy sync");
    return ok ? MG_OK : MG_ERR_HIP;
}

void *mg_unet_stream(const mg_unet *U) { return U ? (void *)U->stream : nullptr; }

int32_t mg_unet_step(const mg_unet *U) { return U ? U->step : 0; }

mg_status mg_unet_set_params(mg_unet *U, const float *host, int64_t count) {
    if (!U || !host || count != U->np) {
        set_error("mg_unet_set_params: null argument or wrong count");
        return MG_ERR_ARG;
    }
    hipStream_t s = U->stream;
    const size_t fb = U->np * sizeof(float);
    bool ok = hip_ok(hipMemcpyAsync(U->p, host, fb, hipMemcpyHostToDevice, s), "parameter upload") &&
              hip_ok(hipStreamSynchronize(s), "parameter upload sync") && mg::nn::fill_f32(U->m, U->np, s) &&
              mg::nn::fill_f32(U->v, U->np, s) && mg::nn::fill_f32(U->g, U->np, s) && refresh_weights(U) &&
              hip_ok(hipStreamSynchronize(s), "parameter refresh");
    U->step = 0;
    return ok ? MG_OK : MG_ERR_HIP;
}

static mg_status download(mg_unet *U, const float *src, float *host, int64_t count, const char *what) {
    if (!U || !host || count != U->np) {
        set_error(std::string(what) + ": null argument or wrong count");
        return MG_ERR_ARG;
    }
    bool ok = hip_ok(hipMemcpyAsync(host, src, U->np * sizeof(float), hipMemcpyDeviceToHost, U->stream), what) &&
              hip_ok(hipStreamSynchronize(U->stream), what);
    return ok ? MG_OK : MG_ERR_HIP;
}

mg_status mg_unet_get_params(mg_unet *U, float *host, int64_t count) {
    return download(U, U ? U->p : nullptr, host, count, "mg_unet_get_params");
}

mg_status mg_unet_get_grads(mg_unet *U, float *host, int64_t count) {
    return download(U, U ? U->g : nullptr, host, count, "mg_unet_get_grads");
}

mg_status mg_unet_loss_grad(mg_unet *U, int32_t n, const double *rho, const int8_t *mask, const double *dirichlet,
                            const double *phi_target, int32_t nx, int32_t ny, int32_t nz, double *loss_out) {
    return loss_grad(U, n, rho, mask, dirichlet, phi_target, nx, ny, nz, loss_out, true);
}

mg_status mg_unet_train_step(mg_unet *U, int32_t n, const double *rho, const int8_t *mask, const double *dirichlet,
                             const double *phi_target, int32_t nx, int32_t ny, int32_t nz, float lr,
                             float weight_decay, double *loss_out) {
    if (!(lr > 0.f) || weight_decay < 0.f) {
        set_error("mg_unet_train_step: lr must be > 0 and weight_decay >= 0");
        return MG_ERR_ARG;
    }
    const mg_status st = loss_grad(U, n, rho, mask, dirichlet, phi_target, nx, ny, nz, nullptr, false);
    if (st != MG_OK) return st;
    U->step++;
    bool ok = mg::nn::adamw(U->p, U->pb, U->g, U->m, U->v, U->np, lr, 0.9f, 0.999f, 1e-8f, weight_decay, U->step,
                            U->stream) &&
              refresh_weights(U);
    if (!ok) return MG_ERR_HIP;
    if (loss_out) {
        if (!hip_ok(hipMemcpyAsync(U->loss_host, U->loss_dev, sizeof(double), hipMemcpyDeviceToHost, U->stream),
                    "loss readback") ||
            !hip_ok(hipStreamSynchronize(U->stream), "loss readback sync"))
            return MG_ERR_HIP;
        *loss_out = *U->loss_host;
    }
    return MG_OK;
}

mg_status mg_unet_infer(mg_unet *U, const double *rho, const int8_t *mask, const double *dirichlet, int32_t nx,
                        int32_t ny, int32_t nz, int32_t stride, double *phi0) {
    if (!U || !rho || !mask || !phi0 || !shape_ok(1, nx, ny, nz, stride)) {
        set_error("mg_unet_infer: invalid arguments (stride 1, 2, 4 or 8; dims multiples of 8 * stride)");
        return MG_ERR_ARG;
    }
    const int cx = nx / stride, cy = ny / stride, cz = nz / stride;
    if (!ensure_workspace(U, 1, cz, cy, cx, false) || !ensure_stats(U, 1)) return MG_ERR_ALLOC;
    hipStream_t s = U->stream;
    const long long vc = (long long)cx * cy * cz;
    if (!mg::nn::stats(rho, mask, (long long)nx * ny * nz, 1, U->st, s) ||
        !mg::nn::pack(rho, mask, dirichlet, U->st, stride, 1, cz, cy, cx, U->x0, s) || !forward(U))
        return MG_ERR_HIP;
    if (stride == 1) {
        return mg::nn::head(U->act[D1B], U->p + U->head_w, U->p + U->head_b, U->st, mask, phi0, vc, 1, s)
                   ? MG_OK
                   : MG_ERR_HIP;
    }
    if (!ensure_f64(U, U->yc, U->yc_len, vc) ||
        !ensure_f64(U, U->up_tmp[0], U->up_len[0], vc * 8) ||
        (stride > 2 && !ensure_f64(U, U->up_tmp[1], U->up_len[1], vc * 64)))
        return MG_ERR_ALLOC;
    if (!mg::nn::head(U->act[D1B], U->p + U->head_w, U->p + U->head_b, U->st, nullptr, U->yc, vc, 1, s))
        return MG_ERR_HIP;
    const double *src = U->yc;
    int dz = cz, dy = cy, dx = cx, k = 0;
    while (dz < nz) {
        const bool last = 2 * dz == nz;
        double *dst = last ? phi0 : U->up_tmp[k];
        if (!mg::nn::up2(src, dst, 1, dz, dy, dx, last ? mask : nullptr, s)) return MG_ERR_HIP;
        src = dst;
        k ^= 1;
        dz *= 2, dy *= 2, dx *= 2;
    }
    return MG_OK;
}

mg_status mg_coarsen_problem(const double *rho, const int8_t *mask, const double *dirichlet, int32_t nx, int32_t ny,
                             int32_t nz, int32_t stride, double *rho_c, int8_t *mask_c, double *dirichlet_c,
                             void *stream) {
    if (!rho || !mask || !rho_c || !mask_c || (dirichlet && !dirichlet_c) || stride < 2 || nx <= 0 || ny <= 0 ||
        nz <= 0 || nx % stride || ny % stride || nz % stride) {
        set_error("mg_coarsen_problem: invalid arguments");
        return MG_ERR_ARG;
    }
    return mg::nn::coarsen(rho, mask, dirichlet, stride, nz / stride, ny / stride, nx / stride, rho_c, mask_c,
                           dirichlet ? dirichlet_c : nullptr, (hipStream_t)stream)
               ? MG_OK
               : MG_ERR_HIP;
}

mg_status mg_upsample_guess(const double *phi_c, int32_t nxc, int32_t nyc, int32_t nzc, const int8_t *mask,
                            double *phi, void *stream) {
    if (!phi_c || !mask || !phi || nxc <= 0 || nyc <= 0 || nzc <= 0) {
        set_error("mg_upsample_guess: invalid arguments");
        return MG_ERR_ARG;
    }
    return mg::nn::up2(phi_c, phi, 1, nzc, nyc, nxc, mask, (hipStream_t)stream) ? MG_OK : MG_ERR_HIP;
}

mg_status mg_unet_save(mg_unet *U, const char *path) {
    if (!U || !path) {
        set_error("mg_unet_save: null argument");
        return MG_ERR_ARG;
    }
    std::vector<float> buf(3 * U->np);
    mg_status st = download(U, U->p, buf.data(), U->np, "mg_unet_save");
    if (st == MG_OK) st = download(U, U->m, buf.data() + U->np, U->np, "mg_unet_save");
    if (st == MG_OK) st = download(U, U->v, buf.data() + 2 * U->np, U->np, "mg_unet_save");
    if (st != MG_OK) return st;
    const long long nb = U->np * 4;
    char hdr[1024];
    snprintf(hdr, sizeof hdr,
             "{\"__metadata__\":{\"format\":\"pt\",\"model\":\"mg-unet-16-32-64-128\",\"step\":\"%d\"},"
             "\"adam_m\":{\"dtype\":\"F32\",\"shape\":[%lld],\"data_offsets\":[%lld,%lld]},"
             "\"adam_v\":{\"dtype\":\"F32\",\"shape\":[%lld],\"data_offsets\":[%lld,%lld]},"
             "\"params\":{\"dtype\":\"F32\",\"shape\":[%lld],\"data_offsets\":[%lld,%lld]}}",
             U->step, U->np, nb, 2 * nb, U->np, 2 * nb, 3 * nb, U->np, 0LL, nb);
    std::string h(hdr);
    while (h.size() % 8) h.push_back(' ');
    FILE *f = fopen(path, "wb");
    if (!f) {
        set_error(std::string("mg_unet_save: cannot open ") + path);
        return MG_ERR_ARG;
    }
    const uint64_t hl = h.size();
    unsigned char le[8];
    for (int i = 0; i < 8; i++) le[i] = (unsigned char)(hl >> (8 * i));
    bool ok = fwrite(le, 1, 8, f) == 8 && fwrite(h.data(), 1, h.size(), f) == h.size() &&
              fwrite(buf.data(), 4, buf.size(), f) == buf.size();
    ok &= fclose(f) == 0;
    if (!ok) {
        set_error(std::string("mg_unet_save: write failed for ") + path);
        return MG_ERR_ARG;
    }
    return MG_OK;
}

mg_status mg_unet_load(mg_unet *U, const char *path) {
    if (!U || !path) {
        set_error("mg_unet_load: null argument");
        return MG_ERR_ARG;
    }
    FILE *f = fopen(path, "rb");
    if (!f) {
        set_error(std::string("mg_unet_load: cannot open ") + path);
        return MG_ERR_ARG;
    }
    auto fail = [&](const std::string &msg) {
        fclose(f);
        set_error("mg_unet_load: " + msg);
        return MG_ERR_ARG;
    };
    unsigned char le[8];
    if (fread(le, 1, 8, f) != 8) return fail("short file");
    uint64_t hl = 0;
    for (int i = 0; i < 8; i++) hl |= (uint64_t)le[i] << (8 * i);
    if (hl == 0 || hl > (1u << 24)) return fail("bad header length");
    std::string hdr(hl, ' ');
    if (fread(&hdr[0], 1, hl, f) != hl) return fail("short header");
    const long long nb = U->np * 4;
    std::vector<float> pv(U->np), mv(U->np, 0.f), vv(U->np, 0.f);
    auto read_tensor = [&](const char *name, std::vector<float> &dst, bool required) -> int {
        std::string dtype;
        std::vector<long long> shape;
        long long o0, o1;
        if (!find_tensor(hdr, name, dtype, shape, o0, o1)) return required ? -1 : 0;
        if (dtype != "F32" || shape.size() != 1 || shape[0] != U->np || o1 - o0 != nb) return -1;
        if (fseek(f, (long)(8 + hl + o0), SEEK_SET) != 0) return -1;
        return fread(dst.data(), 4, U->np, f) == (size_t)U->np ? 1 : -1;
    };
    if (read_tensor("params", pv, true) != 1) return fail("missing or mismatched 'params' (F32, one dimension)");
    const int hm = read_tensor("adam_m", mv, false), hv = read_tensor("adam_v", vv, false);
    if (hm < 0 || hv < 0) return fail("mismatched optimizer state");
    fclose(f);
    int step = 0;
    const size_t k = hdr.find("\"step\"");
    if (k != std::string::npos && hm == 1 && hv == 1) {
        const size_t q = hdr.find('"', hdr.find(':', k));
        step = (int)strtol(hdr.c_str() + q + 1, nullptr, 10);
    }
    mg_status st = mg_unet_set_params(U, pv.data(), U->np);
    if (st != MG_OK) return st;
    if (hm == 1 && hv == 1) {
        bool ok = hip_ok(hipMemcpyAsync(U->m, mv.data(), nb, hipMemcpyHostToDevice, U->stream), "moment upload") &&
                  hip_ok(hipMemcpyAsync(U->v, vv.data(), nb, hipMemcpyHostToDevice, U->stream), "moment upload") &&
                  hip_ok(hipStreamSynchronize(U->stream), "moment upload sync");
        if (!ok) return MG_ERR_HIP;
        U->step = step;
    }
    return MG_OK;
}

}  // extern "C"
