// C ABI of the masked multigrid library: hierarchy construction, the
// multigrid iteration as a fixed kernel sequence (replayed as a hipGraph), the
// solve loop with the runtime order switch, and single-step entry points.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "mg_core.h"

namespace mg {

static thread_local std::string g_err;

void set_error(const std::string &s) { g_err = s; }

bool hip_ok(hipError_t e, const char *what) {
    if (e == hipSuccess) return true;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return false;
}

void *dev_alloc(mg_hierarchy *H, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (H->opt.allocator.alloc) {
        p = H->opt.allocator.alloc(bytes, H->opt.allocator.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) H->allocs.push_back(p);
    return p;
}

namespace {

struct Fail {
    mg_status st;
};

#define HIPCHK(call)                                  \
    do {                                              \
        if (!hip_ok((call), #call)) throw Fail{MG_ERR_HIP}; \
    } while (0)

template <typename T>
T *alloc_n(mg_hierarchy *H, size_t n) {
    void *p = dev_alloc(H, n * sizeof(T));
    if (!p) {
        set_error("device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
        throw Fail{MG_ERR_ALLOC};
    }
    return (T *)p;
}

const OrderData &odata(const mg_hierarchy *H, int l, int order) { return H->lev[l].od[l == 0 ? 2 : order]; }

// ---------------------------------------------------------------- build --

// Releases one allocation made through dev_alloc (after the stream is idle).
void dev_free(mg_hierarchy *H, void *p) {
    if (!p) return;
    for (size_t i = 0; i < H->allocs.size(); i++)
        if (H->allocs[i] == p) {
            if (H->opt.allocator.free) H->opt.allocator.free(p, H->opt.allocator.ctx);
            else if (!H->opt.allocator.alloc) (void)hipFree(p);
            H->allocs[i] = H->allocs.back();
            H->allocs.pop_back();
            return;
        }
}

// Active tile list, smoother work items of `depth` planes and their activity
// masks of level l in boundary order `order`, written to od (its diagonals
// and active count are left as they are).
void build_lists(mg_hierarchy *H, int l, int order, int depth, OrderData &od) {
    Level &L = H->lev[l];
    const int nt = L.ntx * L.nty * L.ntz;
    uint8_t *flags = alloc_n<uint8_t>(H, (size_t)nt);
    launch_tile_flags(L, l, order, flags, H->stream);
    std::vector<uint8_t> hf(nt);
    HIPCHK(hipMemcpyAsync(hf.data(), flags, nt, hipMemcpyDeviceToHost, H->stream));
    HIPCHK(hipStreamSynchronize(H->stream));
    dev_free(H, flags);
    std::vector<int> tiles;
    for (int t = 0; t < nt; t++)
        if (hf[t]) tiles.push_back(t);
    // smoother items: on the finest level runs of active tiles along z, cut
    // every depth / TZ tiles; on coarse levels one active tile cut into
    // depth-plane items
    std::vector<Seg> segs;
    for (int ty = 0; ty < L.nty; ty++)
        for (int tx = 0; tx < L.ntx; tx++) {
            int tz = 0;
            while (tz < L.ntz) {
                if (!hf[(tz * L.nty + ty) * L.ntx + tx]) {
                    tz++;
                    continue;
                }
                int t1 = tz;
                if (l == 0) {
                    const int per = depth / TZ;
                    while (t1 < L.ntz && hf[(t1 * L.nty + ty) * L.ntx + tx] && t1 - tz < per) t1++;
                    segs.push_back(Seg{tx * TX, ty * TY, tz * TZ, std::min(L.nz, t1 * TZ)});
                } else {
                    t1 = tz + 1;
                    for (int z = tz * TZ; z < std::min(L.nz, t1 * TZ); z += depth)
                        segs.push_back(Seg{tx * TX, ty * TY, z, std::min(std::min(L.nz, t1 * TZ), z + depth)});
                }
                tz = t1;
            }
        }
    std::sort(segs.begin(), segs.end(), [](const Seg &a, const Seg &b) {
        if (a.z0 != b.z0) return a.z0 < b.z0;
        if (a.y0 != b.y0) return a.y0 < b.y0;
        return a.x0 < b.x0;
    });
    od.depth = depth;
    od.ntiles = (int)tiles.size();
    od.nsegs = (int)segs.size();
    od.tiles = alloc_n<int>(H, std::max<size_t>(1, tiles.size()));
    od.segs = alloc_n<Seg>(H, std::max<size_t>(1, segs.size()));
    if (!tiles.empty())
        HIPCHK(hipMemcpyAsync(od.tiles, tiles.data(), tiles.size() * sizeof(int), hipMemcpyHostToDevice, H->stream));
    if (!segs.empty())
        HIPCHK(hipMemcpyAsync(od.segs, segs.data(), segs.size() * sizeof(Seg), hipMemcpyHostToDevice, H->stream));
    const int npl = depth + 4;
    od.pmask = alloc_n<unsigned long long>(H, std::max<size_t>(1, segs.size() * npl));
    launch_item_masks(L, l, order, od, npl, od.pmask, H->stream);
    od.pmask3 = nullptr;
    if (l == 0 && H->opt.fuse_restrict && !H->opt.fuse_passes) {  // the last finest pre-smoothing pass
        const int npl3 = depth + 6;
        od.pmask3 = alloc_n<unsigned long long>(H, std::max<size_t>(1, segs.size() * npl3));
        launch_item_masks(L, l, order, od, npl3, od.pmask3, H->stream, 3);
    }
    od.pmask2 = nullptr;
    if (H->opt.fuse_passes) {
        const int npl2 = depth + 8;
        od.pmask2 = alloc_n<unsigned long long>(H, std::max<size_t>(1, segs.size() * npl2));
        launch_item_masks(L, l, order, od, npl2, od.pmask2, H->stream, 4);
    }
    std::vector<Seg> s8;
    if (l == 1) {  // whole tiles for the FP64 prolongation pass
        for (int ty = 0; ty < L.nty; ty++)
            for (int tx = 0; tx < L.ntx; tx++)
                for (int tz = 0; tz < L.ntz; tz++)
                    if (hf[(tz * L.nty + ty) * L.ntx + tx])
                        s8.push_back(Seg{tx * TX, ty * TY, tz * TZ, std::min(L.nz, (tz + 1) * TZ)});
        std::sort(s8.begin(), s8.end(), [](const Seg &a, const Seg &b) {
            if (a.z0 != b.z0) return a.z0 < b.z0;
            if (a.y0 != b.y0) return a.y0 < b.y0;
            return a.x0 < b.x0;
        });
        od.nsegs8 = (int)s8.size();
        od.segs8 = alloc_n<Seg>(H, std::max<size_t>(1, s8.size()));
        if (!s8.empty())
            HIPCHK(hipMemcpyAsync(od.segs8, s8.data(), s8.size() * sizeof(Seg), hipMemcpyHostToDevice, H->stream));
        constexpr int npl8 = TZ + 4;
        od.pmask8 = alloc_n<unsigned long long>(H, std::max<size_t>(1, s8.size() * npl8));
        OrderData t = od;
        t.segs = od.segs8;
        t.nsegs = od.nsegs8;
        launch_item_masks(L, l, order, t, npl8, od.pmask8, H->stream);
    }
    // the host vectors staged above (tiles, segs, s8) are the sources of
    // asynchronous copies: wait for them before the vectors go away
    HIPCHK(hipStreamSynchronize(H->stream));
}

// Frees the lists build_lists made (the stream must be idle).
void free_lists(mg_hierarchy *H, OrderData &od) {
    for (void *p : {(void *)od.tiles, (void *)od.segs, (void *)od.pmask, (void *)od.pmask2, (void *)od.pmask3,
                    (void *)od.segs8, (void *)od.pmask8})
        dev_free(H, p);
    od.tiles = nullptr;
    od.segs = nullptr;
    od.pmask = od.pmask2 = od.pmask8 = nullptr;
    od.segs8 = nullptr;
}

mg_status validate_options(const mg_options &o) {
    if (o.n_pre < 0 || o.n_post < 0 || o.n_cycles < 1 || o.n_coarse_sweeps < 0 || o.min_coarse_dim < 1 ||
        o.max_cycles < 0 || (o.precision != MG_FP64 && o.precision != MG_MIXED) || o.bc_order < 0 ||
        o.bc_order > 2 || !(o.eta > 0) || o.first_order_hold < 0 || o.fuse_passes < 0 || o.fuse_passes > 1 ||
        o.fuse_restrict < 0 || o.fuse_restrict > 1) {
        set_error("invalid mg_options");
        return MG_ERR_ARG;
    }
    if (o.n_cycles > 4) {
        set_error("n_cycles above 4 is not supported");
        return MG_ERR_ARG;
    }
    auto coarse_ok = [&](int v) { return !v || depth_supported(2, v) || (v == DEPTH_CUBE && !o.fuse_passes); };
    if (o.tune < 0 || o.tune > 1 || (o.item_depth_fine && !depth_supported(0, o.item_depth_fine)) ||
        !coarse_ok(o.item_depth_l1) || !coarse_ok(o.item_depth_coarse)) {
        set_error("invalid tune or item depth (finest: 8, 16, 32; coarse: 2, 4, 8, or 1 for cubes "
                  "without fuse_passes)");
        return MG_ERR_ARG;
    }
    if (o.fuse_passes && o.item_depth_fine && o.item_depth_fine != SEG_TILES_FINE * TZ) {
        set_error("fuse_passes runs 16-plane finest work items only");
        return MG_ERR_ARG;
    }
    return MG_OK;
}

// ------------------------------------------------------------- tuning --

// Item depth of level l fixed by the options (0: default or tuned).
int forced_depth(const mg_options &o, int l) {
    return l == 0 ? o.item_depth_fine : l == 1 ? o.item_depth_l1 : o.item_depth_coarse;
}

// March depth a level's lists start with (cube items keep the default march
// for the passes that apply the prolongation).
int start_depth(const mg_options &o, int l) {
    const int f = forced_depth(o, l);
    return (f && f != DEPTH_CUBE) ? f : item_depth(l);
}

// The tuning cache: lines "<key> <depth>" in the file MG_TUNE_CACHE names.
std::string tune_key(const mg_hierarchy *H, int l, int order, bool f32) {
    const Level &L = H->lev[l];
    char b[160];
    snprintf(b, sizeof b, "gfx950:%dx%dx%d:l%d:o%d:%s:a%lld%s", H->lev[0].nx, H->lev[0].ny, H->lev[0].nz, l, order,
             f32 ? "fp32" : "fp64", (long long)L.od[l == 0 ? 2 : order].nact,
             l == 0 && H->opt.fuse_restrict && !H->opt.fuse_passes ? ":res" : "");
    return b;
}

int tune_cache_get(const std::string &key) {
    const char *path = getenv("MG_TUNE_CACHE");
    if (!path || !*path) return 0;
    FILE *fp = fopen(path, "r");
    if (!fp) return 0;
    char k[200];
    int d = 0, found = 0;
    while (fscanf(fp, "%199s %d", k, &d) == 2)
        if (key == k) found = d;  // the last entry wins
    fclose(fp);
    return found;
}

void tune_cache_put(const std::string &key, int depth) {
    const char *path = getenv("MG_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *fp = fopen(path, "a");
    if (!fp) return;
    fprintf(fp, "%s %d\n", key.c_str(), depth);
    fclose(fp);
}

// Average time of the work a cycle runs over the work items of od on
// level l, with HIP events on the hierarchy's stream (best of three runs):
// on coarse levels one smoother pass; on the finest level, which runs
// several kernels over the same items, a plain pass, the pass with the
// residual and its restriction (or a plain pass and the residual march with
// the restriction) and the pass forming its input's norm (FP64) or the
// update with the outer residual (mixed).  At creation every iterate and
// right-hand side buffer holds zeros, which this work keeps; it costs the
// same on any values.
float time_pass(mg_hierarchy *H, int l, int order, const OrderData &od, bool f32) {
    Level &L = H->lev[l];
    const bool coarse = H->nlev[2] > 1;
    // a coarse level with a coarser one restricts after every other pass
    // (on cubes inside the pass itself)
    const bool restricts = l > 0 && l + 1 < H->nlev[order];
    auto pass = [&](int p) {
        if (restricts && (p & 1)) {
            Level &C = H->lev[l + 1];
            if (od.cube) {
                if (f32) launch_rbgs_restrict32(L, C, order, od, L.x32[p & 1], L.x32[(p & 1) ^ 1], L.f32, C.f32,
                                                H->stream);
                else launch_rbgs_restrict(L, C, order, od, L.x[p & 1], L.x[(p & 1) ^ 1], L.f, C.f, H->stream);
            } else if (f32) {
                HIPCHK(launch_rbgs32(L, l, od, L.x32[p & 1], L.x32[(p & 1) ^ 1], L.f32, H->stream));
                launch_restrict32(L, C, l, order, L.x32[(p & 1) ^ 1], L.f32, C.f32, H->stream);
            } else {
                HIPCHK(launch_rbgs(L, l, od, L.x[p & 1], L.x[(p & 1) ^ 1], L.f, H->stream));
                launch_restrict(L, C, l, order, L.x[(p & 1) ^ 1], L.f, C.f, H->stream);
            }
            return;
        }
        if (l == 0 && coarse && od.pmask3 && (p & 1)) {  // the pass that also restricts
            Level &C = H->lev[1];
            if (f32) HIPCHK(launch_rbgs_res_fine32(L, C, 2, od, L.x32[1], L.x32[0], L.f32, C.f32, H->stream));
            else HIPCHK(launch_rbgs_res_fine(L, C, 2, od, L.x[1], L.x[0], L.f, C.f, H->stream));
        } else if (f32) HIPCHK(launch_rbgs32(L, l, od, L.x32[p & 1], L.x32[(p & 1) ^ 1], L.f32, H->stream));
        else HIPCHK(launch_rbgs(L, l, od, L.x[p & 1], L.x[(p & 1) ^ 1], L.f, H->stream));
        if (l != 0 || (p & 1) == 0) return;
        if (f32) {
            if (coarse && !od.pmask3) launch_restrict32(L, H->lev[1], 0, 2, L.x32[0], L.f32, H->lev[1].f32, H->stream);
            launch_axpy_resnorm32(L, od, L.x[0], L.x32[0], L.x[1], L.f, L.f32, H->part, H->norm_dev, 0, H->stream,
                                  nullptr);
        } else {
            if (coarse && !od.pmask3) launch_restrict(L, H->lev[1], 0, 2, L.x[0], L.f, H->lev[1].f, H->stream);
            HIPCHK(launch_rbgs_norm(L, od, L.x[0], L.x[1], L.f, H->part, H->stream));
        }
    };
    // the restriction march reads the finest lists from the level itself
    const OrderData saved = L.od[2];
    if (l == 0) L.od[2] = od;
    const int n = l == 0 ? 10 : 20;
    for (int p = 0; p < 4; p++) pass(p);
    float best = 1e30f;
    for (int rep = 0; rep < 3; rep++) {
        HIPCHK(hipEventRecord(H->ev0, H->stream));
        for (int p = 0; p < n; p++) pass(p);
        HIPCHK(hipEventRecord(H->ev1, H->stream));
        HIPCHK(hipEventSynchronize(H->ev1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, H->ev0, H->ev1));
        best = std::min(best, ms);
    }
    L.od[2] = saved;
    return best / n;
}

// Picks the planes per work item of every level and order that its
// smoother passes run fastest with (each candidate timed on this
// hierarchy), unless the options fix it; levels run by the one-workgroup
// kernel take no work items.  The precision timed is the one the level's
// passes run in (FP32 for a mixed-precision hierarchy).
void tune_depths(mg_hierarchy *H) {
    const bool f32 = H->opt.precision == MG_MIXED;
    for (int l = 0; l < std::max(H->nlev[1], H->nlev[2]); l++)
        for (int o = 2; o >= 1; o--) {
            if (l == 0 && o == 1) continue;  // the finest level is the same in both orders
            if (l >= H->nlev[o] || (H->ls[o] >= 0 && l >= H->ls[o])) continue;
            if (forced_depth(H->opt, l) || (l == 0 && H->opt.fuse_passes)) continue;
            OrderData &od = H->lev[l].od[o];
            if (od.nsegs == 0) continue;
            const std::string key = tune_key(H, l, o, f32);
            int best = tune_cache_get(key);
            if (!depth_supported(l, best) && !(l > 0 && best == DEPTH_CUBE && !H->opt.fuse_passes)) {
                const int cand0[3] = {8, 16, 32}, cand1[3] = {2, 4, 8};
                const int *cand = l == 0 ? cand0 : cand1;
                float tbest = time_pass(H, l, o, od, f32);
                best = od.depth;
                for (int c = 0; c < 3; c++) {
                    if (cand[c] == od.depth) continue;
                    OrderData t = od;
                    build_lists(H, l, o, cand[c], t);
                    const float tc = time_pass(H, l, o, t, f32);
                    HIPCHK(hipStreamSynchronize(H->stream));
                    if (tc < tbest) {
                        tbest = tc;
                        best = cand[c];
                    }
                    free_lists(H, t);
                }
                if (l > 0 && !H->opt.fuse_passes) {  // whole 8^3 cubes instead of a march
                    OrderData t = od;
                    t.cube = true;
                    if (time_pass(H, l, o, t, f32) < tbest) best = DEPTH_CUBE;
                }
                tune_cache_put(key, best);
            }
            const int march = best == DEPTH_CUBE ? od.depth : best;
            if (march != od.depth) {
                HIPCHK(hipStreamSynchronize(H->stream));
                free_lists(H, od);
                build_lists(H, l, o, march, od);
            }
            od.cube = best == DEPTH_CUBE;
        }
    H->lev[0].od[1] = H->lev[0].od[2];
}

void create(mg_hierarchy *H, const int8_t *mask, int nx, int ny, int nz, double h) {
    hipStream_t s = H->stream;
    HIPCHK(hipGetDevice(&H->device));
    // geometry of the levels: halve while every edge is even and stays >= min_coarse_dim
    Level *lev = H->lev;
    lev[0].nx = nx; lev[0].ny = ny; lev[0].nz = nz; lev[0].h = h;
    int L = 1;
    while (L < MAXL) {
        const Level &p = lev[L - 1];
        if (p.nx % 2 || p.ny % 2 || p.nz % 2) break;
        const int m = H->opt.min_coarse_dim;
        if (p.nx / 2 < m || p.ny / 2 < m || p.nz / 2 < m) break;
        lev[L].nx = p.nx / 2; lev[L].ny = p.ny / 2; lev[L].nz = p.nz / 2; lev[L].h = 2 * p.h;
        L++;
    }
    H->nlev_geom = L;
    for (int l = 0; l < L; l++) {
        Level &v = lev[l];
        v.n = (size_t)v.nx * v.ny * v.nz;
        v.ntx = (v.nx + TX - 1) / TX;
        v.nty = (v.ny + TY - 1) / TY;
        v.ntz = (v.nz + TZ - 1) / TZ;
    }
    // validation on the device: bad values, non-inactive frame, active count
    unsigned long long *ctr = alloc_n<unsigned long long>(H, 3 + 2 * MAXL + 1);
    HIPCHK(hipMemsetAsync(ctr, 0, (3 + 2 * MAXL + 1) * sizeof(unsigned long long), s));
    launch_validate(mask, nx, ny, nz, ctr, s);
    unsigned long long hv[3 + 2 * MAXL + 1];
    HIPCHK(hipMemcpyAsync(hv, ctr, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hv[0]) {
        set_error("mask holds " + std::to_string(hv[0]) + " values other than +1/-1");
        throw Fail{MG_ERR_ARG};
    }
    if (hv[1]) {
        set_error("mask has " + std::to_string(hv[1]) + " active cells in the outermost layer");
        throw Fail{MG_ERR_ARG};
    }
    if (hv[2] == 0) {
        set_error("mask has no active cell");
        throw Fail{MG_ERR_NO_ACTIVE};
    }
    // integer mask counts per level (R1 of the mask)
    for (int l = 0; l < L; l++) lev[l].cnt = alloc_n<int32_t>(H, lev[l].n);
    launch_count0(mask, lev[0].cnt, lev[0].n, s);
    for (int l = 1; l < L; l++) launch_count_up(lev[l - 1], lev[l], s);
    // finest code, coarse diagonals per order
    lev[0].code = alloc_n<uint8_t>(H, lev[0].n);
    unsigned long long *nact = ctr + 3;
    launch_code0(lev[0], nact, s);
    for (int o = 1; o <= 2; o++)
        for (int l = 1; l < L; l++) {
            lev[l].od[o].d = alloc_n<double>(H, lev[l].n);
            launch_diag(lev[l], l, o, lev[l].od[o].d, nact + 2 * l + (o - 1), s);
        }
    HIPCHK(hipMemcpyAsync(hv, nact, (2 * MAXL + 1) * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    lev[0].od[1].nact = lev[0].od[2].nact = (int64_t)hv[0];
    for (int o = 1; o <= 2; o++) {
        H->nlev[o] = 1;
        for (int l = 1; l < L; l++) {
            lev[l].od[o].nact = (int64_t)hv[2 * l + (o - 1)];
            if (lev[l].od[o].nact > 0 && H->nlev[o] == l) H->nlev[o] = l + 1;
        }
    }
    // active tile lists and work items (default or fixed depths; tuned below)
    build_lists(H, 0, 2, start_depth(H->opt, 0), lev[0].od[2]);
    lev[0].od[1] = lev[0].od[2];
    for (int o = 1; o <= 2; o++)
        for (int l = 1; l < H->nlev[o]; l++) {
            build_lists(H, l, o, start_depth(H->opt, l), lev[l].od[o]);
            lev[l].od[o].cube = forced_depth(H->opt, l) == DEPTH_CUBE;
        }
    // level buffers
    const int nl = std::max(H->nlev[1], H->nlev[2]);
    const bool mixed = H->opt.precision == MG_MIXED;
    for (int l = 0; l < nl; l++) {
        Level &v = lev[l];
        for (int b = 0; b < 2; b++) {
            v.x[b] = alloc_n<double>(H, v.n);
            HIPCHK(hipMemsetAsync(v.x[b], 0, v.n * sizeof(double), s));
        }
        v.f = alloc_n<double>(H, v.n);
        HIPCHK(hipMemsetAsync(v.f, 0, v.n * sizeof(double), s));
        if (mixed) {
            for (int b = 0; b < 2; b++) {
                v.x32[b] = alloc_n<float>(H, v.n);
                HIPCHK(hipMemsetAsync(v.x32[b], 0, v.n * sizeof(float), s));
            }
            v.f32 = alloc_n<float>(H, v.n);
            HIPCHK(hipMemsetAsync(v.f32, 0, v.n * sizeof(float), s));
            if (l > 0)
                for (int o = 1; o <= 2; o++)
                    if (l < H->nlev[o]) {
                        v.od[o].d32 = alloc_n<float>(H, v.n);
                        launch_to_float(v.od[o].d, v.od[o].d32, v.n, s);
                    }
        }
    }
    // first level of the one-workgroup kernel, per order
    const int small_lim = small_init();
    for (int o = 1; o <= 2; o++) {
        H->ls[o] = -1;
        for (int l = 1; l < H->nlev[o]; l++)
            if (lev[l].n <= SMALL_MAX_CELLS && H->nlev[o] - l <= MAXS &&
                small_lds_bytes(H, o, l, false) <= (size_t)small_lim) {
                H->ls[o] = l;
                break;
            }
        // a deepest level above that size (an edge that stops halving early)
        // still goes to the workgroup when it fits its LDS: its n_coarse
        // sweeps are then one launch instead of one launch each
        const int last = H->nlev[o] - 1;
        if (H->ls[o] < 0 && last >= 1 && small_lds_bytes(H, o, last, false) <= (size_t)small_lim) H->ls[o] = last;
    }
    H->part_cap = std::max(1, lev[0].od[2].ntiles * TZ);
    H->part = alloc_n<double>(H, (size_t)H->part_cap);
    H->norm_dev = alloc_n<double>(H, 8);
    H->halt_dev = alloc_n<int>(H, 1);
    HIPCHK(hipMemsetAsync(H->halt_dev, 0, sizeof(int), s));
    H->stop_dev = alloc_n<StopTest>(H, 1);
    HIPCHK(hipMemsetAsync(H->stop_dev, 0, sizeof(StopTest), s));
    for (int l = 0; l < MAXL; l++) lev[l].halt = H->halt_dev;
    HIPCHK(hipMemsetAsync(H->norm_dev, 0, 8 * sizeof(double), s));
    HIPCHK(hipHostMalloc((void **)&H->norm_host, 8 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHK(hipHostGetDevicePointer((void **)&H->norm_map, H->norm_host, 0));
    HIPCHK(hipEventCreate(&H->ev0));
    HIPCHK(hipEventCreate(&H->ev1));
    for (int q = 0; q < 2; q++) HIPCHK(hipEventCreateWithFlags(&H->evq[q], hipEventDisableTiming));
    for (int q = 0; q < 2; q++)
        HIPCHK(hipEventCreateWithFlags(&H->evn[q], hipEventDisableTiming | hipEventDisableSystemFence));
    HIPCHK(hipStreamSynchronize(s));
    if (H->opt.tune) tune_depths(H);
    HIPCHK(hipStreamSynchronize(s));
    H->coarse_order_state = 0;
}

// ---------------------------------------------------------- iteration --

struct Cur {
    int c[MAXL];
};

// The residual norm of a cycle's input formed by its first finest pass
// (launch_rbgs_norm), its final sum right after that pass (with `stop`, the
// device stop test), which also stores the sum to `host` (device address of
// coherent host memory), followed by `ev`.
struct InputNorm {
    const StopTest *stop;
    double *host;
    hipEvent_t ev;
};

// Kinds of finest-level launch that mg_kernel_timing can record.
enum { KT_PLAIN = 1, KT_RESIDUAL = 2, KT_PROLONG = 3, KT_NORM = 4 };

// Events for the next launch of timing kind `kind`, if the hierarchy records
// that kind and has a pair left (else both null and false).
bool kt_events(mg_hierarchy *H, int kind, hipEvent_t &e0, hipEvent_t &e1) {
    e0 = e1 = nullptr;
    if (H->kt_on != kind || H->kt_used * 2 >= (int)H->kt_ev.size()) return false;
    e0 = H->kt_ev[2 * H->kt_used];
    e1 = H->kt_ev[2 * H->kt_used + 1];
    return true;
}

// `passes` red-black passes on level l; zero_start: the iterate starts at 0.
// in (finest level, FP64, single passes): the first pass also forms the
// residual norm of its input.
void smooth(mg_hierarchy *H, int l, int order, int passes, bool zero_start, Cur &cur, bool f32,
            const InputNorm *in = nullptr) {
    Level &L = H->lev[l];
    const OrderData &od = odata(H, l, order);
    if (passes == 0) {
        if (zero_start) {
            if (f32) launch_zero_tiles32(L, od, L.x32[cur.c[l]], H->stream);
            else launch_zero_tiles(L, od, L.x[cur.c[l]], H->stream);
        }
        return;
    }
    // with fuse_passes each pair of passes is one launch (one buffer flip)
    for (int p = 0; p < passes;) {
        const int a = cur.c[l], b = a ^ 1;
        const bool zin = (p == 0 && zero_start);
        if (in && p == 0 && l == 0 && !f32 && !zin) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            const bool timed = od.nsegs > 0 && kt_events(H, KT_NORM, e0, e1);
            HIPCHK(launch_rbgs_norm(L, od, L.x[a], L.x[b], L.f, H->part, H->stream, e0, e1));
            if (timed) H->kt_used++;
            launch_finalize(L, H->part, od.nsegs, H->norm_dev, 0, in->stop, H->stream, in->host);
            if (in->host) HIPCHK(hipEventRecord(in->ev, H->stream));
            p += 1;
        } else if (H->opt.fuse_passes && passes - p >= 2) {
            if (f32) launch_rbgs2_32(L, l, od, zin ? nullptr : L.x32[a], L.x32[b], L.f32, H->stream);
            else launch_rbgs2(L, l, od, zin ? nullptr : L.x[a], L.x[b], L.f, H->stream);
            p += 2;
        } else {
            // optional timing: the kernel's own start and end on a pair of events
            hipEvent_t e0 = nullptr, e1 = nullptr;
            const bool timed = l == 0 && od.nsegs > 0 && kt_events(H, KT_PLAIN, e0, e1);
            if (f32) HIPCHK(launch_rbgs32(L, l, od, zin ? nullptr : L.x32[a], L.x32[b], L.f32, H->stream, e0, e1));
            else HIPCHK(launch_rbgs(L, l, od, zin ? nullptr : L.x[a], L.x[b], L.f, H->stream, e0, e1));
            if (timed) H->kt_used++;
            p += 1;
        }
        cur.c[l] = b;
    }
}

// Launches (= buffer flips) of `passes` passes.
int pass_launches(const mg_hierarchy *H, int passes) {
    return H->opt.fuse_passes ? passes / 2 + passes % 2 : passes;
}

// One multigrid iteration at level l (Sec. 2 enumerated recipe): N_pre
// passes, residual and R1 restriction, N_cycles iterations of the coarse
// correction problem from zero, P2 prolongation and correction, N_post passes.
// The deepest level is relaxed n_coarse_sweeps times.
void mg_level(mg_hierarchy *H, int l, int order, bool zero_start, Cur &cur, bool f32,
              const InputNorm *in = nullptr) {
    const mg_options &o = H->opt;
    const int last = H->nlev[order] - 1;
    Level &L = H->lev[l];
    if (l == H->ls[order]) {
        // the whole call MG(l) on the small levels in one workgroup
        if (f32) launch_small32(H, order, l, zero_start, L.f32, L.x32[cur.c[l]], H->stream);
        else launch_small(H, order, l, zero_start, L.f, L.x[cur.c[l]], H->stream);
        return;
    }
    if (l == last) {
        smooth(H, l, order, o.n_coarse_sweeps, zero_start, cur, f32);
        return;
    }
    Level &C = H->lev[l + 1];
    const OrderData &odl = odata(H, l, order);
    if (l == 0 && odl.pmask3 && !o.fuse_passes && o.n_pre >= 1 && (o.n_pre >= 2 || !in)) {
        // the last pre-smoothing pass also forms the residual and restricts it
        // (the first pass may have to form the norm of its input instead)
        if (o.n_pre > 1) smooth(H, l, order, o.n_pre - 1, zero_start, cur, f32, in);
        const bool zin = zero_start && o.n_pre == 1;
        const int a = cur.c[l], b = a ^ 1;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const bool timed = odl.nsegs > 0 && kt_events(H, KT_RESIDUAL, e0, e1);
        if (f32)
            HIPCHK(launch_rbgs_res_fine32(L, C, order, odl, zin ? nullptr : L.x32[a], L.x32[b], L.f32, C.f32,
                                          H->stream, e0, e1));
        else
            HIPCHK(launch_rbgs_res_fine(L, C, order, odl, zin ? nullptr : L.x[a], L.x[b], L.f, C.f, H->stream, e0,
                                        e1));
        if (timed) H->kt_used++;
        cur.c[l] = b;
    } else if (l > 0 && odl.cube && o.n_pre >= 1) {
        // cube levels: the last pre-smoothing pass also restricts the residual
        if (o.n_pre > 1) smooth(H, l, order, o.n_pre - 1, zero_start, cur, f32, in);
        const bool zin = zero_start && o.n_pre == 1;
        const int a = cur.c[l], b = a ^ 1;
        if (f32) launch_rbgs_restrict32(L, C, order, odl, zin ? nullptr : L.x32[a], L.x32[b], L.f32, C.f32, H->stream);
        else launch_rbgs_restrict(L, C, order, odl, zin ? nullptr : L.x[a], L.x[b], L.f, C.f, H->stream);
        cur.c[l] = b;
    } else {
        smooth(H, l, order, o.n_pre, zero_start, cur, f32, in);
        if (f32) launch_restrict32(L, C, l, order, L.x32[cur.c[l]], L.f32, C.f32, H->stream);
        else launch_restrict(L, C, l, order, L.x[cur.c[l]], L.f, C.f, H->stream);
    }
    for (int c = 0; c < o.n_cycles; c++) mg_level(H, l + 1, order, c == 0, cur, f32);
    if (o.n_post == 0) {
        if (f32) launch_prolong32(L, C, l, order, C.x32[cur.c[l + 1]], L.x32[cur.c[l]], H->stream);
        else launch_prolong(L, C, l, order, C.x[cur.c[l + 1]], L.x[cur.c[l]], H->stream);
        return;
    }
    // the first post-smoothing pass applies the prolongation as it loads x
    // (on the finest level with fuse_passes, fused with the pass after it)
    const OrderData &od = odata(H, l, order);
    const int a = cur.c[l], b = a ^ 1;
    const bool fused = H->opt.fuse_passes && l == 0 && o.n_post >= 2;
    if (fused) {
        if (f32) launch_rbgs2_prolong32(L, od, C, C.x32[cur.c[l + 1]], L.x32[a], L.x32[b], L.f32, H->stream);
        else launch_rbgs2_prolong(L, od, C, C.x[cur.c[l + 1]], L.x[a], L.x[b], L.f, H->stream);
    } else {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const bool timed = l == 0 && od.nsegs > 0 && kt_events(H, KT_PROLONG, e0, e1);
        if (f32)
            HIPCHK(launch_rbgs_prolong32(L, l, od, C, C.x32[cur.c[l + 1]], L.x32[a], L.x32[b], L.f32, H->stream, e0,
                                         e1));
        else
            HIPCHK(launch_rbgs_prolong(L, l, od, C, C.x[cur.c[l + 1]], L.x[a], L.x[b], L.f, H->stream, e0, e1));
        if (timed) H->kt_used++;
    }
    cur.c[l] = b;
    smooth(H, l, order, o.n_post - (fused ? 2 : 1), false, cur, f32);
}

// Coarse iterates must be 0 outside the active tiles of the order in use.
void ensure_coarse_clean(mg_hierarchy *H, int order) {
    if (H->coarse_order_state == 0 || H->coarse_order_state == order) {
        H->coarse_order_state = order;
        return;
    }
    for (int l = 1; l < std::max(H->nlev[1], H->nlev[2]); l++) {
        Level &L = H->lev[l];
        for (int b = 0; b < 2; b++) {
            HIPCHK(hipMemsetAsync(L.x[b], 0, L.n * sizeof(double), H->stream));
            if (L.x32[b]) HIPCHK(hipMemsetAsync(L.x32[b], 0, L.n * sizeof(float), H->stream));
        }
    }
    H->coarse_order_state = order;
}

void zero_level_x(mg_hierarchy *H, int l) {
    Level &L = H->lev[l];
    for (int b = 0; b < 2; b++) HIPCHK(hipMemsetAsync(L.x[b], 0, L.n * sizeof(double), H->stream));
}

// One solve-loop cycle as a kernel sequence: FP64 MG(0) then the residual
// norm of the new iterate, or (mixed) the FP32 inner MG(0) on L e = f - L x
// from e = 0, x += e, and the FP64 residual norm that also writes the next
// inner right-hand side.  decide: the norm's final sum also runs the stop
// test on the device and sets the halt flag that makes every kernel of a
// following cycle return at once.  FP64 modes: NORM_AFTER as above;
// NORM_INPUT: no norm after the cycle, its first finest pass forms the norm
// of its input (the previous cycle's iterate) as `in` describes; NORM_NONE:
// no norm at all.
enum { NORM_AFTER = 0, NORM_INPUT = 1, NORM_NONE = 2 };

void enqueue_cycle(mg_hierarchy *H, int order, int parity, bool mixed, int *parity_out, bool decide,
                   int mode = NORM_AFTER, const InputNorm *in = nullptr, double *host_out = nullptr) {
    const StopTest *stop = decide ? H->stop_dev : nullptr;
    Cur cur;
    for (int l = 0; l < MAXL; l++) cur.c[l] = 0;
    Level &L0 = H->lev[0];
    const OrderData &od0 = odata(H, 0, order);
    if (!mixed) {
        cur.c[0] = parity;
        mg_level(H, 0, order, false, cur, false, mode == NORM_INPUT ? in : nullptr);
        if (mode == NORM_AFTER)
            launch_resnorm(L0, 0, od0, L0.x[cur.c[0]], L0.f, H->part, H->norm_dev, 0, H->stream, stop, host_out);
    } else {
        mg_level(H, 0, order, true, cur, true);
        // x + e goes to the other FP64 buffer (unused by the FP32 inner cycle)
        launch_axpy_resnorm32(L0, od0, L0.x[parity], L0.x32[cur.c[0]], L0.x[parity ^ 1], L0.f, L0.f32, H->part,
                              H->norm_dev, 0, H->stream, stop, host_out);
    }
    *parity_out = mixed ? parity ^ 1 : cur.c[0];
}

int cycle_parity_after(const mg_hierarchy *H, int order, int parity) {
    const mg_options &o = H->opt;
    int flips;
    if (H->nlev[order] == 1) flips = pass_launches(H, o.n_coarse_sweeps);
    else if (o.n_post == 0) flips = pass_launches(H, o.n_pre);
    else if (o.fuse_passes && o.n_post >= 2) flips = pass_launches(H, o.n_pre) + 1 + pass_launches(H, o.n_post - 2);
    else flips = pass_launches(H, o.n_pre) + 1 + pass_launches(H, o.n_post - 1);
    return parity ^ (flips & 1);
}

void run_cycle_kernels(mg_hierarchy *H, int order, int parity, bool mixed, int *parity_out, bool decide) {
    if (!H->opt.use_graph) {
        enqueue_cycle(H, order, parity, mixed, parity_out, decide);
        return;
    }
    for (auto &g : H->graphs)
        if (g.order == order && g.parity == parity && g.mixed == mixed && g.decide == decide) {
            HIPCHK(hipGraphLaunch(g.exec, H->stream));
            *parity_out = mixed ? parity ^ 1 : cycle_parity_after(H, order, parity);
            return;
        }
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(H->stream, hipStreamCaptureModeThreadLocal));
    try {
        enqueue_cycle(H, order, parity, mixed, parity_out, decide);
    } catch (...) {
        hipGraph_t tmp;
        (void)hipStreamEndCapture(H->stream, &tmp);
        if (tmp) (void)hipGraphDestroy(tmp);
        throw;
    }
    HIPCHK(hipStreamEndCapture(H->stream, &graph));
    Graph g;
    g.order = order;
    g.parity = parity;
    g.mixed = mixed;
    g.decide = decide;
    HIPCHK(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    H->graphs.push_back(g);
    HIPCHK(hipGraphLaunch(g.exec, H->stream));
}

// One cycle whose norm lands in norm_host[host_slot]: launched directly, its
// final sum stores the norm there itself (wait on an evn event); replayed
// from its captured graph (use_graph), followed by an 8-byte copy (wait on
// an evq event).
void run_cycle(mg_hierarchy *H, int order, int parity, bool mixed, int *parity_out, bool decide, int host_slot) {
    if (!H->opt.use_graph) {
        enqueue_cycle(H, order, parity, mixed, parity_out, decide, NORM_AFTER, nullptr, H->norm_map + host_slot);
        return;
    }
    run_cycle_kernels(H, order, parity, mixed, parity_out, decide);
    HIPCHK(hipMemcpyAsync(H->norm_host + host_slot, H->norm_dev, sizeof(double), hipMemcpyDeviceToHost, H->stream));
}

double read_norm(mg_hierarchy *H) {
    HIPCHK(hipStreamSynchronize(H->stream));
    return sqrt(H->norm_host[0]);
}

// The solve loop in phases, so that many hierarchies sharing a stream can
// advance together with one host synchronisation per cycle (batch.hip):
// begin (fold, two reference norms) | start (after a sync) | cycle enqueue |
// cycle finish (after a sync) | end (store).
// Host part of begin: the solve state, the boundary order of this solve and
// the coarse buffers cleaned for it.
void solve_init(mg_hierarchy *H, double *phi, double tol, mg_solve_info *info, SolveState &S) {
    const mg_options &o = H->opt;
    memset(info, 0, sizeof(*info));
    info->switched_at_cycle = -1;
    S = SolveState{};
    S.info = info;
    S.phi = phi;
    S.tol = tol;
    if (o.bc_order == MG_BC_FIRST || o.bc_order == MG_BC_SECOND) {
        S.order = o.bc_order;
    } else if (H->hold_left > 0) {
        S.order = 1;
        H->hold_left--;
    } else {
        S.order = 2;
    }
    S.mixed = o.precision == MG_MIXED;
    ensure_coarse_clean(H, S.order);
}

void solve_begin(mg_hierarchy *H, const double *rho, double *phi, const double *B, double tol, mg_solve_info *info,
                 SolveState &S) {
    solve_init(H, phi, tol, info, S);
    Level &L0 = H->lev[0];
    const OrderData &od0 = odata(H, 0, S.order);
    hipStream_t s = H->stream;
    HIPCHK(hipEventRecord(H->ev0, s));
    launch_set_halt(H->halt_dev, 0, s);
    launch_fold(L0, od0, rho, B, phi, L0.f, L0.x[0], s);
    launch_resnorm(L0, 0, od0, nullptr, L0.f, H->part, H->norm_dev, 1, s);
    if (S.mixed) launch_resnorm32(L0, od0, L0.x[0], L0.f, L0.f32, H->part, H->norm_dev, 0, s);
    else launch_resnorm(L0, 0, od0, L0.x[0], L0.f, H->part, H->norm_dev, 0, s);
    HIPCHK(hipMemcpyAsync(H->norm_host, H->norm_dev, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
}

// After the stream has been synchronised: the reference norms.
void solve_start(mg_hierarchy *H, SolveState &S) {
    mg_solve_info *info = S.info;
    S.rprev = sqrt(H->norm_host[0]);
    S.rref = sqrt(H->norm_host[1]);
    info->r0 = S.rprev;
    if (S.rref == 0.0) S.rref = S.rprev;
    info->r_ref = S.rref;
    info->history[0] = S.rprev;
    info->order_used = S.order;
    info->r_final = S.rprev;
    S.st = MG_NOT_CONVERGED;
    S.parity = 0;
    S.n = 0;
    S.active = true;
    if (!(S.rprev > S.tol * S.rref)) {
        S.st = std::isfinite(S.rprev) ? MG_OK : MG_ERR_DIVERGED;
        S.active = false;
    } else if (H->opt.max_cycles < 1) {
        S.active = false;
    }
}

void solve_cycle_enqueue(mg_hierarchy *H, SolveState &S) {
    int np = S.parity;
    run_cycle(H, S.order, S.parity, S.mixed, &np, false, 0);
    S.host_slot = 0;
    S.parity = np;
}

// After the stream has been synchronised: stop test and order switch (Sec. 4).
void solve_cycle_finish(mg_hierarchy *H, SolveState &S) {
    const mg_options &o = H->opt;
    mg_solve_info *info = S.info;
    const int n = ++S.n;
    const double rn = sqrt(H->norm_host[S.host_slot]);
    info->cycles = n;
    info->r_final = rn;
    if (n < 257) info->history[n] = rn;
    if (!std::isfinite(rn)) {
        S.st = MG_ERR_DIVERGED;
        S.active = false;
        return;
    }
    if (rn <= S.tol * S.rref) {
        S.st = MG_OK;
        S.active = false;
        return;
    }
    if (o.bc_order == MG_BC_AUTO && S.order == 2 && rn / S.rprev > o.eta) {
        S.order = 1;
        H->hold_left = o.first_order_hold;
        info->switched_at_cycle = n;
        info->order_used = 1;
        ensure_coarse_clean(H, S.order);
    }
    S.rprev = rn;
    if (n >= o.max_cycles) S.active = false;
}

void solve_end(mg_hierarchy *H, SolveState &S) {
    Level &L0 = H->lev[0];
    launch_store(L0, odata(H, 0, S.order), L0.x[S.parity], S.phi, H->stream);
    HIPCHK(hipEventRecord(H->ev1, H->stream));
    S.info->status = S.st;
}

// The device copy of the stop test's inputs for the cycles to come.
void set_device_stop(mg_hierarchy *H, const SolveState &S) {
    const bool check = H->opt.bc_order == MG_BC_AUTO && S.order == 2;
    launch_set_stop(H->stop_dev, S.tol * S.rref, S.rprev, H->opt.eta, check ? 1 : 0, H->stream);
}

// One solve with the next cycle always in flight: cycle n+1 is enqueued
// before the host reads cycle n's norm.  Cycle n's norm also runs the stop
// test on the device (the same FP64 comparisons as solve_cycle_finish); if it
// stops or switches order, every kernel of cycle n+1 returns at once and the
// host discards that cycle.  The host's decisions stay authoritative; the GPU
// no longer idles while the host decides.
mg_status solve(mg_hierarchy *H, const double *rho, double *phi, const double *B, double tol, mg_solve_info *info) {
    mg_solve_info tmp;
    if (!info) info = &tmp;
    hipStream_t s = H->stream;
    SolveState S;
    solve_begin(H, rho, phi, B, tol, info, S);
    HIPCHK(hipStreamSynchronize(s));
    solve_start(H, S);
    if (S.active) set_device_stop(H, S);
    const mg_options &o = H->opt;
    if (!S.mixed && !o.use_graph && !o.fuse_passes && o.n_pre >= 1 && H->nlev[1] > 1 && H->nlev[2] > 1) {
        // The norm of cycle k's iterate is formed by the first finest pass of
        // cycle k + 1, so the host decides on it while the rest of cycle k + 1
        // runs; a stop or an order switch halts that rest on the device (its
        // first pass wrote the other buffer only, x_k stays intact).  The last
        // allowed cycle's norm comes from the residual-norm march.
        bool launched = false;  // cycle S.n + 1 is in the stream
        int par_next = S.parity;  // buffer of the iterate of cycle S.n + 1
        int kt_mark = 0;          // timing records before the cycle after S.n + 1
        while (S.active) {
            if (!launched) {
                enqueue_cycle(H, S.order, S.parity, false, &par_next, false, NORM_NONE);
                launched = true;
            }
            const int k = S.n + 1;
            const int slot = 4 + (k & 1);
            int par_after = par_next;
            kt_mark = H->kt_used;
            if (k + 1 <= o.max_cycles) {
                const InputNorm in{H->stop_dev, H->norm_map + slot, H->evn[k & 1]};
                enqueue_cycle(H, S.order, par_next, false, &par_after, true, NORM_INPUT, &in);
            } else {
                Level &L0 = H->lev[0];
                launch_resnorm(L0, 0, odata(H, 0, S.order), L0.x[par_next], L0.f, H->part, H->norm_dev, 0, s,
                               H->stop_dev);
                HIPCHK(hipMemcpyAsync(H->norm_host + slot, H->norm_dev, sizeof(double), hipMemcpyDeviceToHost, s));
                HIPCHK(hipEventRecord(H->evq[k & 1], s));
            }
            HIPCHK(hipEventSynchronize(k + 1 <= o.max_cycles ? H->evn[k & 1] : H->evq[k & 1]));
            const int order_before = S.order;
            S.host_slot = slot;
            solve_cycle_finish(H, S);
            S.parity = par_next;
            if (!S.active || S.order != order_before) {
                // the device stop test halted the rest of cycle k + 1 (its
                // launches returned at once: drop their timing records)
                launched = false;
                H->kt_used = kt_mark;
                if (S.active) {
                    launch_set_halt(H->halt_dev, 0, s);
                    set_device_stop(H, S);
                }
            } else {
                par_next = par_after;  // cycle k + 1 is in flight
            }
        }
        launch_set_halt(H->halt_dev, 0, s);
        solve_end(H, S);
        HIPCHK(hipEventSynchronize(H->ev1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, H->ev0, H->ev1));
        info->ms = ms;
        return S.st;
    }
    struct Flight {
        int parity_out, slot, ev, kt_mark;
    } fl[2];
    int nf = 0, enq = 0, par = S.parity;
    // a directly launched cycle stores its norm to host memory itself
    hipEvent_t *const evc = o.use_graph ? H->evq : H->evn;
    auto launch = [&]() {
        const int k = enq & 1;
        int np = par;
        const int kt_mark = H->kt_used;
        run_cycle(H, S.order, par, S.mixed, &np, true, 4 + k);
        HIPCHK(hipEventRecord(evc[k], s));
        fl[nf++] = Flight{np, 4 + k, k, kt_mark};
        par = np;
        enq++;
    };
    while (S.active) {
        if (nf == 0) launch();
        if (nf == 1 && S.n + 2 <= H->opt.max_cycles) launch();  // speculative
        HIPCHK(hipEventSynchronize(evc[fl[0].ev]));
        const int order_before = S.order;
        S.host_slot = fl[0].slot;
        solve_cycle_finish(H, S);
        S.parity = fl[0].parity_out;
        fl[0] = fl[1];
        nf--;
        if (!S.active || S.order != order_before) {
            // the cycle in flight found the halt flag set and did nothing
            if (nf) {
                HIPCHK(hipEventSynchronize(evc[fl[0].ev]));
                H->kt_used = fl[0].kt_mark;
            }
            nf = 0;
            par = S.parity;
            if (S.active) {
                launch_set_halt(H->halt_dev, 0, s);
                set_device_stop(H, S);
            }
        }
    }
    launch_set_halt(H->halt_dev, 0, s);  // other entry points run with the flag clear
    solve_end(H, S);
    HIPCHK(hipEventSynchronize(H->ev1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, H->ev0, H->ev1));
    info->ms = ms;
    return S.st;
}

mg_status check_level(const mg_hierarchy *H, int level, int order, bool need_coarser) {
    if (!H) {
        set_error("null hierarchy");
        return MG_ERR_ARG;
    }
    if (order != 1 && order != 2) {
        set_error("order must be 1 or 2");
        return MG_ERR_ARG;
    }
    const int top = H->nlev[order] - (need_coarser ? 1 : 0);
    if (level < 0 || level >= top) {
        set_error("level out of range for this order");
        return MG_ERR_ARG;
    }
    return MG_OK;
}

template <class F>
mg_status guarded(F &&fn) {
    try {
        return fn();
    } catch (const Fail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return MG_ERR_ALLOC;
    } catch (...) {
        set_error("unexpected internal error");
        return MG_ERR_HIP;
    }
}

}  // namespace

mg_status phase_begin(mg_hierarchy *H, const double *rho, double *phi, const double *B, double tol,
                      mg_solve_info *info, SolveState &S) {
    return guarded([&]() {
        solve_begin(H, rho, phi, B, tol, info, S);
        return MG_OK;
    });
}

mg_status phase_init(mg_hierarchy *H, double *phi, double tol, mg_solve_info *info, SolveState &S) {
    return guarded([&]() {
        solve_init(H, phi, tol, info, S);
        return MG_OK;
    });
}

mg_status phase_start(mg_hierarchy *H, SolveState &S) {
    return guarded([&]() {
        solve_start(H, S);
        return MG_OK;
    });
}

mg_status phase_cycle_enqueue(mg_hierarchy *H, SolveState &S) {
    return guarded([&]() {
        solve_cycle_enqueue(H, S);
        return MG_OK;
    });
}

mg_status phase_cycle_finish(mg_hierarchy *H, SolveState &S) {
    return guarded([&]() {
        solve_cycle_finish(H, S);
        return MG_OK;
    });
}

mg_status phase_end(mg_hierarchy *H, SolveState &S) {
    return guarded([&]() {
        solve_end(H, S);
        return MG_OK;
    });
}

}  // namespace mg

using namespace mg;

extern "C" {

void mg_default_options(mg_options *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->n_pre = 2;
    o->n_post = 2;
    o->n_cycles = 1;
    o->n_coarse_sweeps = 32;
    o->min_coarse_dim = 4;
    o->max_cycles = 200;
    o->precision = MG_FP64;
    o->bc_order = MG_BC_AUTO;
    o->eta = 0.5;
    o->first_order_hold = 10;
    o->use_graph = 0;
    o->fuse_restrict = 1;
}

const char *mg_status_string(mg_status s) {
    switch (s) {
        case MG_OK: return "ok";
        case MG_NOT_CONVERGED: return "not converged (max_cycles reached)";
        case MG_ERR_ARG: return "invalid argument";
        case MG_ERR_NO_ACTIVE: return "mask has no active cell";
        case MG_ERR_HIP: return "HIP runtime error";
        case MG_ERR_DIVERGED: return "diverged (non-finite residual)";
        case MG_ERR_ALLOC: return "allocation failed";
    }
    return "unknown status";
}

const char *mg_last_error(void) { return g_err.c_str(); }

void mg_destroy_hierarchy(mg_hierarchy *H) {
    if (!H) return;
    for (auto &g : H->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (H->stream) (void)hipStreamSynchronize(H->stream);
    for (void *p : H->allocs) {
        if (H->opt.allocator.free) H->opt.allocator.free(p, H->opt.allocator.ctx);
        else if (!H->opt.allocator.alloc) (void)hipFree(p);
    }
    if (H->norm_host) (void)hipHostFree(H->norm_host);
    if (H->own_stream && H->stream) (void)hipStreamDestroy(H->stream);
    for (hipEvent_t e : H->kt_ev) (void)hipEventDestroy(e);
    if (H->ev0) (void)hipEventDestroy(H->ev0);
    if (H->ev1) (void)hipEventDestroy(H->ev1);
    for (int q = 0; q < 2; q++) {
        if (H->evq[q]) (void)hipEventDestroy(H->evq[q]);
        if (H->evn[q]) (void)hipEventDestroy(H->evn[q]);
    }
    delete H;
}

mg_status mg_create_hierarchy(const int8_t *mask_dev, int32_t nx, int32_t ny, int32_t nz, double h,
                              const mg_options *opt, void *stream, mg_hierarchy **out) {
    set_error("");
    if (!out) {
        set_error("out is NULL");
        return MG_ERR_ARG;
    }
    *out = nullptr;
    if (!mask_dev || nx < 1 || ny < 1 || nz < 1 || !(h > 0) || !std::isfinite(h)) {
        set_error("invalid mask pointer, dims or h");
        return MG_ERR_ARG;
    }
    if ((size_t)nx * ny * nz >= ((size_t)1 << 34) || (size_t)nx * ny * sizeof(double) >= ((size_t)1 << 31)) {
        set_error("box too large (at most 2^34 cells and 2^28 cells per z-plane)");
        return MG_ERR_ARG;
    }
    mg_hierarchy *H = new (std::nothrow) mg_hierarchy();
    if (!H) return MG_ERR_ALLOC;
    if (opt) H->opt = *opt;
    else mg_default_options(&H->opt);
    mg_status st = validate_options(H->opt);
    if (st != MG_OK) {
        delete H;
        return st;
    }
    H->stream = (hipStream_t)stream;
    st = guarded([&]() {
        if (!H->stream) {
            // the legacy null stream cannot be captured into a graph: use a
            // blocking stream of our own (it still orders with the null stream)
            HIPCHK(hipStreamCreate(&H->stream));
            H->own_stream = true;
        }
        create(H, mask_dev, nx, ny, nz, h);
        return MG_OK;
    });
    if (st != MG_OK) {
        mg_destroy_hierarchy(H);
        return st;
    }
    *out = H;
    return MG_OK;
}

mg_status mg_solve(mg_hierarchy *H, const double *rho_dev, double *phi_dev, const double *dirichlet_dev, double tol,
                   mg_solve_info *info) {
    if (!H || !rho_dev || !phi_dev || !(tol > 0)) {
        set_error("null argument or tol <= 0");
        return MG_ERR_ARG;
    }
    return guarded([&]() { return solve(H, rho_dev, phi_dev, dirichlet_dev, tol, info); });
}

mg_status mg_residual_norm(mg_hierarchy *H, const double *rho_dev, const double *phi_dev,
                           const double *dirichlet_dev, double *norm_out) {
    if (!H || !rho_dev || !phi_dev || !norm_out) {
        set_error("null argument");
        return MG_ERR_ARG;
    }
    return guarded([&]() {
        Level &L0 = H->lev[0];
        const OrderData &od0 = odata(H, 0, 2);
        // fold into the hierarchy's own buffers, then ||L x - f||
        launch_fold(L0, od0, rho_dev, dirichlet_dev, phi_dev, L0.f, L0.x[0], H->stream);
        launch_resnorm(L0, 0, od0, L0.x[0], L0.f, H->part, H->norm_dev, 0, H->stream);
        HIPCHK(hipMemcpyAsync(H->norm_host, H->norm_dev, sizeof(double), hipMemcpyDeviceToHost, H->stream));
        *norm_out = read_norm(H);
        return MG_OK;
    });
}

}  // extern "C"

// Scratch of mg_residual_norm_noalloc: the per-item partial sums of squares
// and their total, in a file-scope device array, so that the call allocates
// nothing.  Host code must never pass `scratch` itself to a kernel (in host
// code it names a host-side stand-in): its device address is taken once per
// device with hipGetSymbolAddress and kept in g_scratch_dev.
namespace {

constexpr int NOALLOC_DOUBLES = 1 << 17;   // 1 MiB per device
constexpr int NOALLOC_PART = 64;           // partials start here; [0] holds the total
constexpr int NOALLOC_MAX_DEV = 64;
__device__ __align__(256) double scratch[NOALLOC_DOUBLES];

std::mutex g_scratch_mu;
double *g_scratch_dev[NOALLOC_MAX_DEV] = {};

// Device address of `scratch` on device `dev`, which must be current.
double *scratch_on(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (dev < 0 || dev >= NOALLOC_MAX_DEV) {
        set_error("device index out of range for the static scratch");
        return nullptr;
    }
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        if (!hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)")) return nullptr;
        g_scratch_dev[dev] = (double *)p;
    }
    return g_scratch_dev[dev];
}

__global__ void k_sqrt_out(const double *__restrict__ sq, double *__restrict__ out) { out[0] = sqrt(sq[0]); }

}  // namespace

extern "C" {

mg_status mg_residual_norm_noalloc(mg_hierarchy *H, const double *rho_dev, const double *phi_dev,
                                   const double *dirichlet_dev, double *norm_dev) {
    if (!H || !rho_dev || !phi_dev || !norm_dev) {
        set_error("null argument");
        return MG_ERR_ARG;
    }
    const OrderData &od0 = odata(H, 0, 2);
    if (od0.nsegs > NOALLOC_DOUBLES - NOALLOC_PART) {
        set_error("mg_residual_norm_noalloc: " + std::to_string(od0.nsegs) +
                  " finest work items exceed the static scratch (" + std::to_string(NOALLOC_DOUBLES - NOALLOC_PART) +
                  " partial sums)");
        return MG_ERR_ARG;
    }
    int dev = -1;
    if (!hip_ok(hipGetDevice(&dev), "hipGetDevice")) return MG_ERR_HIP;
    if (dev != H->device) {
        set_error("mg_residual_norm_noalloc: the current device is not the hierarchy's");
        return MG_ERR_ARG;
    }
    double *sc = scratch_on(dev);
    if (!sc) return MG_ERR_HIP;
    return guarded([&]() {
        Level &L0 = H->lev[0];
        // the same kernels as mg_residual_norm; every partial the final sum
        // reads is written by the march of this call, so nothing is cleared
        launch_fold(L0, od0, rho_dev, dirichlet_dev, phi_dev, L0.f, L0.x[0], H->stream);
        launch_resnorm(L0, 0, od0, L0.x[0], L0.f, sc + NOALLOC_PART, sc, 0, H->stream, nullptr);
        k_sqrt_out<<<1, 1, 0, H->stream>>>(sc, norm_dev);
        HIPCHK(hipGetLastError());
        return MG_OK;
    });
}

int32_t mg_num_levels(const mg_hierarchy *H, int32_t order) {
    if (!H) return 0;
    if (order == 1 || order == 2) return H->nlev[order];
    return H->nlev_geom;
}

mg_status mg_level_dims(const mg_hierarchy *H, int32_t level, int32_t *dims_out) {
    if (!H || !dims_out || level < 0 || level >= H->nlev_geom) {
        set_error("invalid level");
        return MG_ERR_ARG;
    }
    dims_out[0] = H->lev[level].nx;
    dims_out[1] = H->lev[level].ny;
    dims_out[2] = H->lev[level].nz;
    return MG_OK;
}

int32_t mg_level_item_depth(const mg_hierarchy *H, int32_t level, int32_t order) {
    if (!H || level < 0 || (order != 1 && order != 2) || level >= H->nlev[order]) return -1;
    const OrderData &od = H->lev[level].od[level == 0 ? 2 : order];
    return od.cube ? DEPTH_CUBE : od.depth;
}

int64_t mg_level_active(const mg_hierarchy *H, int32_t level, int32_t order) {
    if (!H || level < 0 || level >= H->nlev_geom || (order != 1 && order != 2)) return -1;
    return H->lev[level].od[level == 0 ? 2 : order].nact;
}

mg_status mg_level_counts(const mg_hierarchy *H, int32_t level, int32_t *counts_dev) {
    if (!H || !counts_dev || level < 0 || level >= H->nlev_geom) {
        set_error("invalid level or pointer");
        return MG_ERR_ARG;
    }
    return guarded([&]() {
        const Level &L = H->lev[level];
        HIPCHK(hipMemcpyAsync(counts_dev, L.cnt, L.n * sizeof(int32_t), hipMemcpyDeviceToDevice, H->stream));
        HIPCHK(hipStreamSynchronize(H->stream));
        return MG_OK;
    });
}

mg_status mg_level_diag(const mg_hierarchy *H, int32_t level, int32_t order, double *d_dev) {
    if (!H || !d_dev || level < 0 || level >= H->nlev_geom || (order != 1 && order != 2)) {
        set_error("invalid level, order or pointer");
        return MG_ERR_ARG;
    }
    return guarded([&]() {
        const Level &L = H->lev[level];
        if (level == 0) {
            // diagonal of the finest level: the cell code itself (0 if inactive)
            std::vector<uint8_t> code(L.n);
            std::vector<double> d(L.n);
            HIPCHK(hipMemcpyAsync(code.data(), L.code, L.n, hipMemcpyDeviceToHost, H->stream));
            HIPCHK(hipStreamSynchronize(H->stream));
            for (size_t p = 0; p < L.n; p++) d[p] = (double)code[p];
            HIPCHK(hipMemcpyAsync(d_dev, d.data(), L.n * sizeof(double), hipMemcpyHostToDevice, H->stream));
        } else {
            HIPCHK(hipMemcpyAsync(d_dev, L.od[order].d, L.n * sizeof(double), hipMemcpyDeviceToDevice, H->stream));
        }
        HIPCHK(hipStreamSynchronize(H->stream));
        return MG_OK;
    });
}

mg_status mg_fold(mg_hierarchy *H, const double *rho_dev, const double *dirichlet_dev, double *f_dev) {
    if (!H || !rho_dev || !f_dev) {
        set_error("null argument");
        return MG_ERR_ARG;
    }
    return guarded([&]() {
        Level &L0 = H->lev[0];
        HIPCHK(hipMemsetAsync(f_dev, 0, L0.n * sizeof(double), H->stream));
        launch_fold(L0, odata(H, 0, 2), rho_dev, dirichlet_dev, nullptr, f_dev, nullptr, H->stream);
        HIPCHK(hipStreamSynchronize(H->stream));
        return MG_OK;
    });
}

mg_status mg_smooth(mg_hierarchy *H, int32_t level, int32_t order, double *x_dev, const double *f_dev,
                    int32_t passes) {
    mg_status st = check_level(H, level, order, false);
    if (st != MG_OK) return st;
    if (!x_dev || !f_dev || passes < 0) {
        set_error("null argument or negative passes");
        return MG_ERR_ARG;
    }
    return guarded([&]() {
        Level &L = H->lev[level];
        const OrderData &od = odata(H, level, order);
        zero_level_x(H, level);
        launch_copy_masked(L, level, od, x_dev, L.x[0], H->stream);
        int c = 0;
        for (int p = 0; p < passes;) {
            if (H->opt.fuse_passes && passes - p >= 2) {
                launch_rbgs2(L, level, od, L.x[c], L.x[c ^ 1], f_dev, H->stream);
                p += 2;
            } else {
                HIPCHK(launch_rbgs(L, level, od, L.x[c], L.x[c ^ 1], f_dev, H->stream));
                p += 1;
            }
            c ^= 1;
        }
        HIPCHK(hipMemcpyAsync(x_dev, L.x[c], L.n * sizeof(double), hipMemcpyDeviceToDevice, H->stream));
        zero_level_x(H, level);
        HIPCHK(hipStreamSynchronize(H->stream));
        if (level > 0) H->coarse_order_state = 0;
        return MG_OK;
    });
}

mg_status mg_residual(mg_hierarchy *H, int32_t level, int32_t order, const double *x_dev, const double *f_dev,
                      double *r_dev) {
    mg_status st = check_level(H, level, order, false);
    if (st != MG_OK) return st;
    if (!x_dev || !f_dev || !r_dev) {
        set_error("null argument");
        return MG_ERR_ARG;
    }
    return guarded([&]() {
        Level &L = H->lev[level];
        const OrderData &od = odata(H, level, order);
        zero_level_x(H, level);
        launch_copy_masked(L, level, od, x_dev, L.x[0], H->stream);
        HIPCHK(hipMemsetAsync(r_dev, 0, L.n * sizeof(double), H->stream));
        launch_residual(L, level, od, L.x[0], f_dev, r_dev, H->stream);
        zero_level_x(H, level);
        HIPCHK(hipStreamSynchronize(H->stream));
        if (level > 0) H->coarse_order_state = 0;
        return MG_OK;
    });
}

mg_status mg_restrict_residual(mg_hierarchy *H, int32_t level, int32_t order, const double *x_dev,
                               const double *f_dev, double *fc_dev) {
    mg_status st = check_level(H, level, order, true);
    if (st != MG_OK) return st;
    if (!x_dev || !f_dev || !fc_dev) {
        set_error("null argument");
        return MG_ERR_ARG;
    }
    return guarded([&]() {
        Level &L = H->lev[level];
        Level &C = H->lev[level + 1];
        const OrderData &od = odata(H, level, order);
        zero_level_x(H, level);
        launch_copy_masked(L, level, od, x_dev, L.x[0], H->stream);
        HIPCHK(hipMemsetAsync(fc_dev, 0, C.n * sizeof(double), H->stream));
        launch_restrict(L, C, level, order, L.x[0], f_dev, fc_dev, H->stream);
        zero_level_x(H, level);
        HIPCHK(hipStreamSynchronize(H->stream));
        if (level > 0) H->coarse_order_state = 0;
        return MG_OK;
    });
}

mg_status mg_prolong(mg_hierarchy *H, int32_t level, int32_t order, const double *xc_dev, double *x_dev) {
    mg_status st = check_level(H, level, order, true);
    if (st != MG_OK) return st;
    if (!x_dev || !xc_dev) {
        set_error("null argument");
        return MG_ERR_ARG;
    }
    return guarded([&]() {
        Level &L = H->lev[level];
        Level &C = H->lev[level + 1];
        zero_level_x(H, level + 1);
        launch_copy_masked(C, level + 1, odata(H, level + 1, order), xc_dev, C.x[0], H->stream);
        launch_prolong(L, C, level, order, C.x[0], x_dev, H->stream);
        zero_level_x(H, level + 1);
        HIPCHK(hipStreamSynchronize(H->stream));
        H->coarse_order_state = 0;
        return MG_OK;
    });
}

mg_status mg_vcycle(mg_hierarchy *H, int32_t order, double *x_dev, const double *f_dev) {
    mg_status st = check_level(H, 0, order, false);
    if (st != MG_OK) return st;
    if (!x_dev || !f_dev) {
        set_error("null argument");
        return MG_ERR_ARG;
    }
    return guarded([&]() {
        Level &L0 = H->lev[0];
        const OrderData &od0 = odata(H, 0, order);
        ensure_coarse_clean(H, order);
        launch_copy_masked(L0, 0, od0, x_dev, L0.x[0], H->stream);
        HIPCHK(hipMemcpyAsync(L0.f, f_dev, L0.n * sizeof(double), hipMemcpyDeviceToDevice, H->stream));
        Cur cur;
        for (int l = 0; l < MAXL; l++) cur.c[l] = 0;
        mg_level(H, 0, order, false, cur, false);
        launch_store(L0, od0, L0.x[cur.c[0]], x_dev, H->stream);
        HIPCHK(hipStreamSynchronize(H->stream));
        return MG_OK;
    });
}

mg_status mg_time_smoother(mg_hierarchy *H, int32_t order, int32_t launches) {
    if (!H || (order != 1 && order != 2) || launches < 0) {
        set_error("invalid argument");
        return MG_ERR_ARG;
    }
    return guarded([&]() {
        Level &L0 = H->lev[0];
        const OrderData &od0 = odata(H, 0, order);
        for (int p = 0; p < launches; p++) {
            if (H->opt.fuse_passes) launch_rbgs2(L0, 0, od0, L0.x[p & 1], L0.x[(p & 1) ^ 1], L0.f, H->stream);
            else HIPCHK(launch_rbgs(L0, 0, od0, L0.x[p & 1], L0.x[(p & 1) ^ 1], L0.f, H->stream));
        }
        if (launches & 1)
            HIPCHK(hipMemcpyAsync(L0.x[0], L0.x[1], L0.n * sizeof(double), hipMemcpyDeviceToDevice, H->stream));
        return MG_OK;
    });
}

mg_status mg_kernel_timing(mg_hierarchy *H, int32_t enable) {
    if (!H || enable < 0 || enable > 4) {
        set_error("invalid argument");
        return MG_ERR_ARG;
    }
    if (enable && H->opt.use_graph) {
        set_error("mg_kernel_timing: a captured cycle records no events (use_graph is set)");
        return MG_ERR_ARG;
    }
    return guarded([&]() {
        HIPCHK(hipSetDevice(H->device));
        HIPCHK(hipStreamSynchronize(H->stream));  // no recorded pair is still pending
        if (enable && H->kt_ev.empty()) {
            H->kt_ev.assign(2 * KT_MAX_LAUNCHES, nullptr);
            // no system-scope fence: a timed launch then ends with the same
            // device-scope release as an untimed one
            for (hipEvent_t &e : H->kt_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        }
        H->kt_on = enable;
        if (enable) H->kt_used = 0;
        return MG_OK;
    });
}

mg_status mg_kernel_timing_read(mg_hierarchy *H, double *ms_total, int32_t *launches) {
    if (!H || !ms_total || !launches) {
        set_error("invalid argument");
        return MG_ERR_ARG;
    }
    return guarded([&]() {
        HIPCHK(hipStreamSynchronize(H->stream));
        double total = 0.0;
        for (int i = 0; i < H->kt_used; i++) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, H->kt_ev[2 * i], H->kt_ev[2 * i + 1]));
            total += ms;
        }
        *ms_total = total;
        *launches = H->kt_used;
        return MG_OK;
    });
}

void *mg_stream(const mg_hierarchy *H) { return H ? (void *)H->stream : nullptr; }

}  // extern "C"
