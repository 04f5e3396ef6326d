// Batched solver: many independent masked grids (AMR-level patches of uneven
// size and depth) advanced together, one persistent launch per multigrid
// cycle for the whole batch.
//
// Each patch has its own hierarchy (same construction and operators as a
// single solve).  The cycle of Sec. 2 for every patch is flattened on the host
// into a fixed program of phases; a phase is a list of work items of one kind
// (a red-black pass over a 32 x 8 x 8 tile of one patch level, a restriction
// or prolongation over a tile, the small-level call MG(ls) of one patch in one
// workgroup, norm partials over a tile, ...).  One cooperative launch runs the
// phases in order, the blocks taking items of a phase round-robin, with a grid
// barrier between phases.  Patches whose multigrid calls reach a given level
// share that level's phases, so patches of different depths interleave.  The
// barrier spins for a bounded time and reports an error instead of hanging.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "coarse_core.h"
#include "smooth_core.h"
#include "transfer_core.h"

namespace mg {
namespace {

// The persistent cooperative kernel below is switched off: its first GPU runs
// ended in HSA_STATUS_ERROR_MEMORY_APERTURE_VIOLATION (a generic-address
// access out of every aperture) and the faulting access has not been found.
// With it off, mg_solve_batch advances all patches in lockstep: each round
// enqueues one graph-captured cycle (the single-grid path, same kernels and
// results) of every unconverged patch, spread over a few streams, and then
// synchronises once for all of them.
constexpr bool kPersistentEnabled = false;
constexpr int kPatchStreams = 4;  // hardware queues of one process
constexpr int BNT = 256;
constexpr int BSEGZ = TZ;  // batch smoother items are one tile deep
constexpr unsigned long long BARRIER_SPIN_LIMIT = 1ull << 24;

enum : int {
    PH_SMOOTH0 = 0,   // red-black pass, finest level
    PH_SMOOTH = 1,    // red-black pass, coarse level
    PH_RESTRICT0 = 2, // residual + R1 from the finest level
    PH_RESTRICT = 3,  // residual + R1 from a coarse level
    PH_PROLONG0 = 4,  // P2 + correction onto the finest level
    PH_PROLONG = 5,   // P2 + correction onto a coarse level
    PH_SMALL = 6,     // MG(ls) of one patch in one workgroup
    PH_NORM = 7,      // residual-norm partials over a finest tile (flags: 1 = with x)
    PH_NORMSUM = 8,   // per-patch fixed-order sum of its partials into norm2[slot]
    PH_FOLD = 9,      // Dirichlet fold and guess load over a finest tile
    PH_STORE = 10,    // copy the finest iterate back to the caller's phi
};

// Level descriptor of one patch (device copy).
struct PLev {
    int nx, ny, nz, ntx, nty;
    double h2, ih2;
    double *x[2];
    double *f;
    const uint8_t *code;    // finest level only
    const double *d[3];     // coarse diagonals, index = order
};

struct BItem {
    int patch;
    int level;
    int tile;               // tile id, or first partial index (NORMSUM)
    int sel;                // bit 0: input iterate buffer; bit 1: start from zero;
                            // bit 2: coarse buffer (PROLONG); NORMSUM: partial count
    Seg seg;                // smoother work item
};

struct Phase {
    int type, first, count, flags;
};

struct BatchArgs {
    const Phase *ph;
    int nph;
    int npatch;
    const BItem *items;
    const PLev *lev;                       // [npatch * MAXL]
    const small::SmallLevels<double> *sl;  // [npatch]: small levels of this program's order
    double *const *small_scratch;          // [npatch]: global scratch when the small levels exceed LDS
    double *part;                          // norm partials, one per NORM item
    double *norm2;                         // [npatch * 2]
    const int *state;                      // [npatch]: 0 = skip, else the boundary order in use
    int order;                             // order this program serves
    const double *const *rho;              // [npatch] inputs of the solve
    const double *const *dir;
    double *const *phi;
    unsigned *bar;                         // [2]: arrival count, generation
    int *err;
    int n_pre, n_post, n_cycles, n_coarse;
};

union BatchLds {
    rb::RbgsLds<double, true> fine;
    rb::RbgsLds<double, false> coarse;
    double small_levels[sizeof(rb::RbgsLds<double, false>) / sizeof(double)];
};

// Grid-wide barrier for a co-resident (cooperative) launch.  Device-scope
// fences make each phase's writes visible to every XCD before the next phase.
// The wait is bounded: on timeout it raises err and lets the block go on, so
// every wave always reaches the end of the kernel.
__device__ void grid_barrier(unsigned *bar, int *err) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = atomicAdd(&bar[0], 1u) + 1u;
        if (arrived == gridDim.x) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned long long spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > BARRIER_SPIN_LIMIT) {
                    atomicExch(err, 1);
                    break;
                }
            }
        }
        __threadfence();
    }
    __syncthreads();
}

__global__ __launch_bounds__(BNT) void k_batch(BatchArgs A) {
    __shared__ BatchLds lds;
    for (int ph = 0; ph < A.nph; ph++) {
        const Phase P = A.ph[ph];
        for (int it = blockIdx.x; it < P.count; it += gridDim.x) {
            const BItem w = A.items[P.first + it];
            if (w.patch < 0 || w.patch >= A.npatch || w.level < 0 || w.level >= MAXL - 1) continue;
            if (A.state[w.patch] != A.order) continue;  // converged or served by the other order's program
            const PLev &L = A.lev[w.patch * MAXL + w.level];
            switch (P.type) {
                case PH_SMOOTH0:
                case PH_SMOOTH: {
                    const int a = w.sel & 1;
                    const double *xin = (w.sel & 2) ? nullptr : L.x[a];
                    if (P.type == PH_SMOOTH0)
                        rb::rbgs_item<double, true, BSEGZ>(lds.fine, xin, L.x[a ^ 1], L.f, L.code, nullptr, L.nx,
                                                           L.ny, L.nz, L.h2, w.seg, nullptr);
                    else
                        rb::rbgs_item<double, false, BSEGZ>(lds.coarse, xin, L.x[a ^ 1], L.f, nullptr,
                                                            L.d[A.order], L.nx, L.ny, L.nz, L.h2, w.seg, nullptr);
                    __syncthreads();
                    break;
                }
                case PH_RESTRICT0:
                case PH_RESTRICT: {
                    const PLev &C = A.lev[w.patch * MAXL + w.level + 1];
                    const double *x = L.x[w.sel & 1];
                    for (int kk = 0; kk < TZ; kk++) {
                        const tr::TileCoord t = tr::tile_cell(w.tile, kk, C.ntx, C.nty, C.nx, C.ny, C.nz);
                        if (P.type == PH_RESTRICT0)
                            tr::restrict_cell<double, true>(t, C.nx, C.ny, C.d[A.order], L.nx, L.ny, L.nz, L.ih2,
                                                            L.code, nullptr, x, L.f, C.f);
                        else
                            tr::restrict_cell<double, false>(t, C.nx, C.ny, C.d[A.order], L.nx, L.ny, L.nz, L.ih2,
                                                             nullptr, L.d[A.order], x, L.f, C.f);
                    }
                    break;
                }
                case PH_PROLONG0:
                case PH_PROLONG: {
                    const PLev &C = A.lev[w.patch * MAXL + w.level + 1];
                    double *x = L.x[w.sel & 1];
                    const double *xc = C.x[(w.sel >> 2) & 1];
                    for (int q = 0; q < tr::NQ; q++) {
                        const tr::Col c = tr::tile_col(w.tile, q, L.ntx, L.nty, L.nx, L.ny);
                        if (P.type == PH_PROLONG0)
                            tr::prolong_col<double, true>(c, L.nx, L.ny, L.nz, L.code, nullptr, xc, C.nx, C.ny, C.nz,
                                                          x);
                        else
                            tr::prolong_col<double, false>(c, L.nx, L.ny, L.nz, nullptr, L.d[A.order], xc, C.nx,
                                                           C.ny, C.nz, x);
                    }
                    break;
                }
                case PH_SMALL: {
                    double *scratch = A.small_scratch[w.patch];
                    double *sm = scratch ? scratch : lds.small_levels;
                    small::small_tail<double>(sm, A.sl[w.patch], L.f, L.x[w.sel & 1], (w.sel & 2) == 0);
                    break;
                }
                case PH_NORM: {
                    double acc = 0.0;
                    for (int q = 0; q < tr::NQ; q++) {
                        const tr::Col c = tr::tile_col(w.tile, q, L.ntx, L.nty, L.nx, L.ny);
                        if (P.flags & 1)
                            acc += tr::resnorm_col<true, true, false>(c, L.nx, L.ny, L.nz, L.ih2, L.code, nullptr,
                                                                      L.x[w.sel & 1], L.f, nullptr);
                        else
                            acc += tr::resnorm_col<true, false, false>(c, L.nx, L.ny, L.nz, L.ih2, L.code, nullptr,
                                                                       nullptr, L.f, nullptr);
                    }
                    const double s = tr::block_sum(acc);
                    if (threadIdx.x == 0) A.part[P.first + it] = s;
                    break;
                }
                case PH_NORMSUM: {
                    // partials of this patch: part[w.tile .. w.tile + w.sel), summed in order
                    if (threadIdx.x == 0) {
                        double s = 0.0;
                        for (int q = 0; q < w.sel; q++) s += A.part[w.tile + q];
                        A.norm2[w.patch * 2 + (P.flags & 1)] = s;
                    }
                    break;
                }
                case PH_FOLD: {
                    for (int kk = 0; kk < TZ; kk++)
                        tr::fold_cell(tr::tile_cell(w.tile, kk, L.ntx, L.nty, L.nx, L.ny, L.nz), L.nx, L.ny, L.ih2,
                                      L.code, A.rho[w.patch], A.dir[w.patch], A.phi[w.patch], L.f, L.x[0]);
                    break;
                }
                case PH_STORE: {
                    for (int kk = 0; kk < TZ; kk++)
                        tr::store_cell(tr::tile_cell(w.tile, kk, L.ntx, L.nty, L.nx, L.ny, L.nz), L.nx, L.ny, L.code,
                                       L.x[w.sel & 1], A.phi[w.patch]);
                    break;
                }
                default:
                    break;
            }
        }
        if (ph + 1 < A.nph) grid_barrier(A.bar, A.err);
    }
}

}  // namespace
}  // namespace mg

// ------------------------------------------------------------------ host --

struct mg_batch {
    int n = 0;
    mg_options opt;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<mg_hierarchy *> patches;
    // per patch and order: first small level (-1: none, never in a batch)
    std::vector<int> ls[3];
    std::vector<void *> allocs;                   // batch-owned device memory
    mg::PLev *lev = nullptr;                      // device [n * MAXL]
    mg::small::SmallLevels<double> *sl[3] = {};   // device [n], per order
    double **small_scratch[3] = {};               // device [n], per order
    // programs: fold, cycle per order, store
    struct Prog {
        mg::Phase *ph = nullptr;
        int nph = 0;
        mg::BItem *items = nullptr;
        int nitems = 0;
    };
    Prog fold, store, cycle[3];
    std::vector<int> cycle_parity[3];  // finest-level buffer holding x after a cycle from buffer 0
    double *part = nullptr;
    int part_cap = 0;
    double *norm2 = nullptr;      // device [2n]
    double *norm2_host = nullptr; // pinned
    int *state = nullptr;         // device [n]
    const double **in_rho = nullptr, **in_dir = nullptr;
    double **in_phi = nullptr;
    unsigned *bar = nullptr;
    int *err = nullptr;
    int grid = 0;
    std::vector<int> hold;
    // pinned staging of per-solve uploads: input pointers, and one state array
    // per queued program (the host never rewrites a buffer a pending copy reads)
    const double **pin_ptrs = nullptr;  // [3n]: rho, dirichlet, phi
    int *pin_state = nullptr;           // [3n]: fold/store, order 2, order 1
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // lockstep engine: patch p runs on pstreams[p % size]
    std::vector<hipStream_t> pstreams;
    std::vector<hipEvent_t> pevents;
};

namespace mg {
namespace {

struct BFail {
    mg_status st;
};

#define BHIP(call)                                           \
    do {                                                     \
        if (!hip_ok((call), #call)) throw BFail{MG_ERR_HIP}; \
    } while (0)

template <typename T>
T *balloc(mg_batch *B, size_t n) {
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(n * sizeof(T), 256);
    if (B->opt.allocator.alloc) p = B->opt.allocator.alloc(bytes, B->opt.allocator.ctx);
    else if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    if (!p) {
        set_error("batch device allocation failed");
        throw BFail{MG_ERR_ALLOC};
    }
    B->allocs.push_back(p);
    return (T *)p;
}

// Host vectors are temporaries: copy and wait before they go away.
template <typename T>
T *upload(mg_batch *B, const std::vector<T> &v) {
    T *d = balloc<T>(B, v.size());
    if (!v.empty()) {
        BHIP(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, B->stream));
        BHIP(hipStreamSynchronize(B->stream));
    }
    return d;
}

std::vector<int> tiles_of(mg_batch *B, const OrderData &od) {
    std::vector<int> t(od.ntiles);
    if (od.ntiles) {
        BHIP(hipMemcpyAsync(t.data(), od.tiles, od.ntiles * sizeof(int), hipMemcpyDeviceToHost, B->stream));
        BHIP(hipStreamSynchronize(B->stream));
    }
    return t;
}

// Host view of the patch hierarchies used while emitting programs.
struct Planner {
    mg_batch *B;
    int order;
    std::vector<std::vector<int>> tiles[MAXL];  // [level][patch]
    std::vector<std::vector<int>> cur;          // [patch][level] buffer holding the iterate
    std::vector<Phase> ph;
    std::vector<BItem> items;
    int nparts = 0;

    const std::vector<int> &tl(int p, int l) {
        if (tiles[l].empty()) tiles[l].resize(B->n);
        if (tiles[l][p].empty()) {
            const Level &L = B->patches[p]->lev[l];
            tiles[l][p] = tiles_of(B, L.od[l == 0 ? 2 : order]);
            if (tiles[l][p].empty()) tiles[l][p].push_back(-1);  // marker: no tile
        }
        return tiles[l][p];
    }
    void begin(int type, int flags = 0) { ph.push_back(Phase{type, (int)items.size(), 0, flags}); }
    void end() {
        ph.back().count = (int)items.size() - ph.back().first;
        if (ph.back().count == 0) ph.pop_back();
    }
    Seg seg_of(const Level &L, int tile) {
        const int tx = tile % L.ntx, ty = (tile / L.ntx) % L.nty, tz = tile / (L.ntx * L.nty);
        return Seg{tx * TX, ty * TY, tz * TZ, std::min(L.nz, (tz + 1) * TZ)};
    }
    void smooth(const std::vector<int> &ps, int l, bool zero) {
        begin(l == 0 ? PH_SMOOTH0 : PH_SMOOTH);
        for (int p : ps) {
            const Level &L = B->patches[p]->lev[l];
            for (int t : tl(p, l))
                if (t >= 0) items.push_back(BItem{p, l, 0, cur[p][l] | (zero ? 2 : 0), seg_of(L, t)});
        }
        end();
        for (int p : ps) cur[p][l] ^= 1;
    }
    // MG(l) for the patches ps (all have at least l+1 levels in this order)
    void mg(const std::vector<int> &ps, int l, bool zero) {
        const mg_options &o = B->opt;
        std::vector<int> small, reg;
        for (int p : ps) (B->ls[order][p] == l ? small : reg).push_back(p);
        if (!small.empty()) {
            begin(PH_SMALL);
            for (int p : small) items.push_back(BItem{p, l, 0, cur[p][l] | (zero ? 2 : 0), Seg{}});
            end();
        }
        if (reg.empty()) return;
        for (int j = 0; j < o.n_pre; j++) smooth(reg, l, zero && j == 0);
        begin(l == 0 ? PH_RESTRICT0 : PH_RESTRICT);
        for (int p : reg)
            for (int t : tl(p, l + 1))
                if (t >= 0) items.push_back(BItem{p, l, t, cur[p][l], Seg{}});
        end();
        for (int c = 0; c < o.n_cycles; c++) mg(reg, l + 1, c == 0);
        begin(l == 0 ? PH_PROLONG0 : PH_PROLONG);
        for (int p : reg)
            for (int t : tl(p, l))
                if (t >= 0) items.push_back(BItem{p, l, t, cur[p][l] | (cur[p][l + 1] << 2), Seg{}});
        end();
        for (int j = 0; j < o.n_post; j++) smooth(reg, l, false);
    }
    // residual-norm partials of every patch's finest level, then per-patch sums into slot
    void norm(bool with_x, int slot) {
        std::vector<int> first(B->n), count(B->n);
        begin(PH_NORM, with_x ? 1 : 0);
        for (int p = 0; p < B->n; p++) {
            first[p] = (int)items.size();
            for (int t : tl(p, 0))
                if (t >= 0) items.push_back(BItem{p, 0, t, cur[p][0], Seg{}});
            count[p] = (int)items.size() - first[p];
        }
        end();
        nparts = std::max(nparts, (int)items.size());
        begin(PH_NORMSUM, slot);
        for (int p = 0; p < B->n; p++) items.push_back(BItem{p, 0, first[p], count[p], Seg{}});
        end();
    }
};

mg_batch::Prog finish(mg_batch *B, Planner &P) {
    mg_batch::Prog g;
    g.ph = upload(B, P.ph);
    g.nph = (int)P.ph.size();
    g.items = upload(B, P.items);
    g.nitems = (int)P.items.size();
    B->part_cap = std::max(B->part_cap, (int)P.items.size());
    return g;
}

void build_batch(mg_batch *B, const int8_t *const *masks, const int32_t *dims, const double *h) {
    const int n = B->n;
    BHIP(hipEventCreate(&B->ev0));
    BHIP(hipEventCreate(&B->ev1));
    if (!kPersistentEnabled) {
        // patch streams (default priority), ordered after the batch stream
        BHIP(hipEventRecord(B->ev0, B->stream));
        for (int k = 0; k < std::min(n, kPatchStreams); k++) {
            hipStream_t ps = nullptr;
            BHIP(hipStreamCreate(&ps));
            B->pstreams.push_back(ps);
            hipEvent_t ev = nullptr;
            BHIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            B->pevents.push_back(ev);
            BHIP(hipStreamWaitEvent(ps, B->ev0, 0));
        }
    }
    // per-patch hierarchies (their own kernels are not used by the persistent engine)
    B->patches.resize(n, nullptr);
    for (int p = 0; p < n; p++) {
        mg_options o = B->opt;
        o.use_graph = kPersistentEnabled ? 0 : 1;
        mg_hierarchy *H = nullptr;
        void *ps = kPersistentEnabled ? (void *)B->stream : (void *)B->pstreams[p % B->pstreams.size()];
        const mg_status st = mg_create_hierarchy(masks[p], dims[3 * p], dims[3 * p + 1], dims[3 * p + 2], h[p], &o,
                                                 ps, &H);
        if (st != MG_OK) throw BFail{st};
        B->patches[p] = H;
        if (kPersistentEnabled && (H->nlev[1] < 2 || H->nlev[2] < 2)) {
            set_error("batch patch " + std::to_string(p) + " has no coarse level");
            throw BFail{MG_ERR_ARG};
        }
    }
    if (!kPersistentEnabled) {
        for (hipStream_t ps : B->pstreams) BHIP(hipStreamSynchronize(ps));
        BHIP(hipStreamSynchronize(B->stream));
        return;
    }
    // level descriptors
    std::vector<PLev> lev((size_t)n * MAXL);
    for (int p = 0; p < n; p++)
        for (int l = 0; l < B->patches[p]->nlev_geom; l++) {
            const Level &L = B->patches[p]->lev[l];
            PLev &d = lev[(size_t)p * MAXL + l];
            d.nx = L.nx; d.ny = L.ny; d.nz = L.nz; d.ntx = L.ntx; d.nty = L.nty;
            d.h2 = L.h * L.h;
            d.ih2 = 1.0 / (L.h * L.h);
            d.x[0] = L.x[0]; d.x[1] = L.x[1]; d.f = L.f;
            d.code = L.code;
            d.d[1] = L.od[1].d; d.d[2] = L.od[2].d;
        }
    B->lev = upload(B, lev);
    // small levels per patch and order: the first coarse level that fits the
    // kernel's LDS budget, else the deepest level run from global scratch
    const size_t lds_budget = sizeof(BatchLds);
    for (int o = 1; o <= 2; o++) {
        B->ls[o].assign(n, -1);
        std::vector<small::SmallLevels<double>> sl(n);
        std::vector<double *> scr(n, nullptr);
        for (int p = 0; p < n; p++) {
            mg_hierarchy *H = B->patches[p];
            int ls = -1;
            for (int l = 1; l < H->nlev[o]; l++)
                if (H->nlev[o] - l <= MAXS && small_lds_bytes(H, o, l, false) <= lds_budget) {
                    ls = l;
                    break;
                }
            if (ls < 0) {
                ls = std::max(1, H->nlev[o] - MAXS);
                ls = std::max(ls, H->nlev[o] - 1);
                scr[p] = balloc<double>(B, small_lds_bytes(H, o, ls, false) / sizeof(double));
            }
            B->ls[o][p] = ls;
            small::SmallLevels<double> &S = sl[p];
            memset(&S, 0, sizeof(S));
            S.n = H->nlev[o] - ls;
            int off = 0;
            for (int q = 0; q < S.n; q++) {
                const Level &L = H->lev[ls + q];
                S.nx[q] = L.nx; S.ny[q] = L.ny; S.nz[q] = L.nz;
                S.mx[q] = small::div_magic((unsigned)L.nx);
                S.mxy[q] = small::div_magic((unsigned)(L.nx * L.ny));
                S.mh[q] = small::div_magic((unsigned)((L.nx + 1) / 2));
                S.mhy[q] = small::div_magic((unsigned)((L.nx + 1) / 2 * L.ny));
                S.h2[q] = L.h * L.h;
                S.ih2[q] = 1.0 / (L.h * L.h);
                S.d[q] = L.od[o].d;
                S.off[q] = off;
                off += 3 * (int)L.n;
            }
            S.n_pre = B->opt.n_pre;
            S.n_post = B->opt.n_post;
            S.n_cycles = B->opt.n_cycles;
            S.n_coarse = B->opt.n_coarse_sweeps;
        }
        B->sl[o] = upload(B, sl);
        B->small_scratch[o] = upload(B, scr);
    }
    // programs
    for (int o = 1; o <= 2; o++) {
        Planner P{B, o};
        P.cur.assign(n, std::vector<int>(MAXL, 0));
        std::vector<int> all(n);
        for (int p = 0; p < n; p++) all[p] = p;
        P.mg(all, 0, false);
        P.norm(true, 0);
        B->cycle_parity[o].resize(n);
        for (int p = 0; p < n; p++) B->cycle_parity[o][p] = P.cur[p][0];
        B->cycle[o] = finish(B, P);
    }
    {
        Planner P{B, 2};
        P.cur.assign(n, std::vector<int>(MAXL, 0));
        P.begin(PH_FOLD);
        for (int p = 0; p < n; p++)
            for (int t : P.tl(p, 0))
                if (t >= 0) P.items.push_back(BItem{p, 0, t, 0, Seg{}});
        P.end();
        P.norm(false, 1);
        P.norm(true, 0);
        B->fold = finish(B, P);
    }
    B->part = balloc<double>(B, (size_t)B->part_cap);
    B->norm2 = balloc<double>(B, 2 * (size_t)n);
    BHIP(hipHostMalloc((void **)&B->norm2_host, 2 * (size_t)n * sizeof(double), hipHostMallocDefault));
    B->state = balloc<int>(B, n);
    B->in_rho = (const double **)balloc<double *>(B, n);
    B->in_dir = (const double **)balloc<double *>(B, n);
    B->in_phi = balloc<double *>(B, n);
    B->bar = balloc<unsigned>(B, 2);
    B->err = balloc<int>(B, 1);
    BHIP(hipMemsetAsync(B->bar, 0, 2 * sizeof(unsigned), B->stream));
    BHIP(hipMemsetAsync(B->err, 0, sizeof(int), B->stream));
    // co-resident grid for the cooperative launch
    int dev = 0, ncu = 0, per = 0;
    BHIP(hipGetDevice(&dev));
    BHIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    BHIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)k_batch, BNT, 0));
    if (per < 1) {
        set_error("batch kernel cannot be resident");
        throw BFail{MG_ERR_HIP};
    }
    B->grid = ncu * per;
    B->hold.assign(n, 0);
    BHIP(hipHostMalloc((void **)&B->pin_ptrs, 3 * (size_t)n * sizeof(double *), hipHostMallocDefault));
    BHIP(hipHostMalloc((void **)&B->pin_state, 3 * (size_t)n * sizeof(int), hipHostMallocDefault));
    BHIP(hipStreamSynchronize(B->stream));
}

void run_program(mg_batch *B, const mg_batch::Prog &g, int order) {
    BatchArgs A;
    memset(&A, 0, sizeof(A));
    A.ph = g.ph;
    A.nph = g.nph;
    A.npatch = B->n;
    A.items = g.items;
    A.lev = B->lev;
    A.sl = B->sl[order];
    A.small_scratch = B->small_scratch[order];
    A.part = B->part;
    A.norm2 = B->norm2;
    A.state = B->state;
    A.order = order;
    A.rho = B->in_rho;
    A.dir = B->in_dir;
    A.phi = B->in_phi;
    A.bar = B->bar;
    A.err = B->err;
    A.n_pre = B->opt.n_pre;
    A.n_post = B->opt.n_post;
    A.n_cycles = B->opt.n_cycles;
    A.n_coarse = B->opt.n_coarse_sweeps;
    void *args[] = {&A};
    BHIP(hipLaunchCooperativeKernel((const void *)k_batch, dim3(B->grid), dim3(BNT), args, 0, B->stream));
}

void check_barrier(mg_batch *B) {
    int e = 0;
    BHIP(hipMemcpyAsync(&e, B->err, sizeof(int), hipMemcpyDeviceToHost, B->stream));
    BHIP(hipStreamSynchronize(B->stream));
    if (e) {
        set_error("batch grid barrier timed out (blocks not co-resident)");
        throw BFail{MG_ERR_HIP};
    }
}

void clean_coarse(mg_batch *B, int p) {
    mg_hierarchy *H = B->patches[p];
    for (int l = 1; l < std::max(H->nlev[1], H->nlev[2]); l++)
        for (int b = 0; b < 2; b++)
            BHIP(hipMemsetAsync(H->lev[l].x[b], 0, H->lev[l].n * sizeof(double), B->stream));
}

// Batch solve on the single-grid path in lockstep: every round enqueues one
// cycle of each unconverged patch (its captured graph and 8-byte norm copy)
// on the patch's stream, then synchronises all patch streams once and
// applies each patch's stop test and order switch (Sec. 2, Sec. 4).
mg_status solve_batch_lockstep(mg_batch *B, const double *const *rho, double *const *phi, const double *const *dir,
                               double tol, mg_solve_info *infos, double *ms_out) {
    const int n = B->n;
    std::vector<mg_solve_info> tmp;
    if (!infos) {
        tmp.resize(n);
        infos = tmp.data();
    }
    std::vector<SolveState> S(n);
    auto sync_all = [&]() {
        for (hipStream_t ps : B->pstreams) BHIP(hipStreamSynchronize(ps));
    };
    BHIP(hipEventRecord(B->ev0, B->stream));
    for (hipStream_t ps : B->pstreams) BHIP(hipStreamWaitEvent(ps, B->ev0, 0));
    for (int p = 0; p < n; p++) {
        const mg_status st = phase_begin(B->patches[p], rho[p], phi[p], dir ? dir[p] : nullptr, tol, &infos[p], S[p]);
        if (st != MG_OK) return st;
    }
    sync_all();
    for (int p = 0; p < n; p++) {
        const mg_status st = phase_start(B->patches[p], S[p]);
        if (st != MG_OK) return st;
    }
    std::vector<int> run;
    while (true) {
        run.clear();
        for (int p = 0; p < n; p++)
            if (S[p].active) run.push_back(p);
        if (run.empty()) break;
        for (int p : run) {
            const mg_status st = phase_cycle_enqueue(B->patches[p], S[p]);
            if (st != MG_OK) return st;
        }
        sync_all();
        for (int p : run) {
            const mg_status st = phase_cycle_finish(B->patches[p], S[p]);
            if (st != MG_OK) return st;
        }
    }
    for (int p = 0; p < n; p++) {
        const mg_status st = phase_end(B->patches[p], S[p]);
        if (st != MG_OK) return st;
    }
    for (size_t k = 0; k < B->pstreams.size(); k++) {
        BHIP(hipEventRecord(B->pevents[k], B->pstreams[k]));
        BHIP(hipStreamWaitEvent(B->stream, B->pevents[k], 0));
    }
    BHIP(hipEventRecord(B->ev1, B->stream));
    BHIP(hipEventSynchronize(B->ev1));
    float ms = 0.f;
    BHIP(hipEventElapsedTime(&ms, B->ev0, B->ev1));
    if (ms_out) *ms_out = ms;
    mg_status worst = MG_OK;
    for (int p = 0; p < n; p++) {
        infos[p].ms = ms;
        const mg_status st = S[p].st;
        if (st < 0 || (st == MG_NOT_CONVERGED && worst == MG_OK)) worst = st;
    }
    return worst;
}

mg_status solve_batch(mg_batch *B, const double *const *rho, double *const *phi, const double *const *dir, double tol,
                      mg_solve_info *infos, double *ms_out) {
    if (!kPersistentEnabled) return solve_batch_lockstep(B, rho, phi, dir, tol, infos, ms_out);
    const int n = B->n;
    const mg_options &o = B->opt;
    std::vector<mg_solve_info> tmp;
    if (!infos) {
        tmp.resize(n);
        infos = tmp.data();
    }
    std::vector<int> order(n), st(n, MG_NOT_CONVERGED), parity(n, 0), active(n, 1);
    std::vector<double> rref(n), rprev(n);
    for (int p = 0; p < n; p++) {
        memset(&infos[p], 0, sizeof(mg_solve_info));
        infos[p].switched_at_cycle = -1;
        if (o.bc_order == MG_BC_FIRST || o.bc_order == MG_BC_SECOND) order[p] = o.bc_order;
        else if (B->hold[p] > 0) {
            order[p] = 1;
            B->hold[p]--;
        } else order[p] = 2;
        if (B->patches[p]->coarse_order_state != 0 && B->patches[p]->coarse_order_state != order[p]) clean_coarse(B, p);
        B->patches[p]->coarse_order_state = order[p];
    }
    BHIP(hipStreamSynchronize(B->stream));  // no copy of an earlier solve still reads the staging
    const double **pr = B->pin_ptrs, **pd = B->pin_ptrs + n, **pp = B->pin_ptrs + 2 * n;
    int *s_all = B->pin_state, *s_ord[3] = {nullptr, B->pin_state + 2 * n, B->pin_state + n};
    for (int p = 0; p < n; p++) {
        pr[p] = rho[p];
        pd[p] = dir ? dir[p] : nullptr;
        pp[p] = phi[p];
        s_all[p] = 2;
    }
    BHIP(hipEventRecord(B->ev0, B->stream));
    BHIP(hipMemsetAsync(B->bar, 0, 2 * sizeof(unsigned), B->stream));
    BHIP(hipMemsetAsync(B->err, 0, sizeof(int), B->stream));
    BHIP(hipMemcpyAsync((void *)B->in_rho, pr, n * sizeof(double *), hipMemcpyHostToDevice, B->stream));
    BHIP(hipMemcpyAsync((void *)B->in_dir, pd, n * sizeof(double *), hipMemcpyHostToDevice, B->stream));
    BHIP(hipMemcpyAsync((void *)B->in_phi, pp, n * sizeof(double *), hipMemcpyHostToDevice, B->stream));
    BHIP(hipMemcpyAsync(B->state, s_all, n * sizeof(int), hipMemcpyHostToDevice, B->stream));
    run_program(B, B->fold, 2);
    BHIP(hipMemcpyAsync(B->norm2_host, B->norm2, 2 * n * sizeof(double), hipMemcpyDeviceToHost, B->stream));
    check_barrier(B);
    for (int p = 0; p < n; p++) {
        const double r0 = sqrt(B->norm2_host[2 * p]);
        double rf = sqrt(B->norm2_host[2 * p + 1]);
        if (rf == 0.0) rf = r0;
        rref[p] = rf;
        rprev[p] = r0;
        infos[p].r0 = r0;
        infos[p].r_ref = rf;
        infos[p].history[0] = r0;
        infos[p].r_final = r0;
        infos[p].order_used = order[p];
        if (!(r0 > tol * rf)) {
            st[p] = std::isfinite(r0) ? MG_OK : MG_ERR_DIVERGED;
            active[p] = 0;
        }
    }
    for (int cyc = 1; cyc <= o.max_cycles; cyc++) {
        bool any = false;
        for (int p = 0; p < n; p++) any |= active[p] != 0;
        if (!any) break;
        for (int oo = 2; oo >= 1; oo--) {
            int *sv = s_ord[oo];  // previous cycle's copies finished (synchronised below)
            bool use = false;
            for (int p = 0; p < n; p++) {
                sv[p] = (active[p] && order[p] == oo) ? oo : 0;
                use |= sv[p] != 0;
            }
            if (!use) continue;
            BHIP(hipMemcpyAsync(B->state, sv, n * sizeof(int), hipMemcpyHostToDevice, B->stream));
            run_program(B, B->cycle[oo], oo);
        }
        BHIP(hipMemcpyAsync(B->norm2_host, B->norm2, 2 * n * sizeof(double), hipMemcpyDeviceToHost, B->stream));
        check_barrier(B);
        for (int p = 0; p < n; p++) {
            if (!active[p]) continue;
            parity[p] = B->cycle_parity[order[p]][p] ^ parity[p];
            const double rn = sqrt(B->norm2_host[2 * p]);
            infos[p].cycles = cyc;
            infos[p].r_final = rn;
            if (cyc < 257) infos[p].history[cyc] = rn;
            if (!std::isfinite(rn)) {
                st[p] = MG_ERR_DIVERGED;
                active[p] = 0;
                continue;
            }
            if (rn <= tol * rref[p]) {
                st[p] = MG_OK;
                active[p] = 0;
                continue;
            }
            if (o.bc_order == MG_BC_AUTO && order[p] == 2 && rn / rprev[p] > o.eta) {
                order[p] = 1;
                B->hold[p] = o.first_order_hold;
                infos[p].switched_at_cycle = cyc;
                infos[p].order_used = 1;
                clean_coarse(B, p);
                B->patches[p]->coarse_order_state = 1;
            }
            rprev[p] = rn;
        }
    }
    // store every patch's iterate (s_all still holds 2 for every patch)
    BHIP(hipMemcpyAsync(B->state, s_all, n * sizeof(int), hipMemcpyHostToDevice, B->stream));
    run_program(B, B->store, 2);
    BHIP(hipEventRecord(B->ev1, B->stream));
    check_barrier(B);
    float ms = 0.f;
    BHIP(hipEventElapsedTime(&ms, B->ev0, B->ev1));
    if (ms_out) *ms_out = ms;
    mg_status worst = MG_OK;
    for (int p = 0; p < n; p++) {
        infos[p].status = st[p];
        infos[p].ms = ms;
        if (st[p] < 0 || (st[p] == MG_NOT_CONVERGED && worst == MG_OK)) worst = (mg_status)st[p];
    }
    return worst;
}

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" {

void mg_destroy_batch(mg_batch *B) {
    if (!B) return;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    for (hipStream_t ps : B->pstreams) (void)hipStreamSynchronize(ps);
    for (mg_hierarchy *H : B->patches) mg_destroy_hierarchy(H);
    for (hipEvent_t ev : B->pevents) (void)hipEventDestroy(ev);
    for (hipStream_t ps : B->pstreams) (void)hipStreamDestroy(ps);
    for (void *p : B->allocs) {
        if (B->opt.allocator.free) B->opt.allocator.free(p, B->opt.allocator.ctx);
        else if (!B->opt.allocator.alloc) (void)hipFree(p);
    }
    if (B->norm2_host) (void)hipHostFree(B->norm2_host);
    if (B->pin_ptrs) (void)hipHostFree((void *)B->pin_ptrs);
    if (B->pin_state) (void)hipHostFree(B->pin_state);
    if (B->ev0) (void)hipEventDestroy(B->ev0);
    if (B->ev1) (void)hipEventDestroy(B->ev1);
    if (B->own_stream && B->stream) (void)hipStreamDestroy(B->stream);
    delete B;
}

mg_status mg_create_batch(int32_t n, const int8_t *const *masks_dev, const int32_t *dims, const double *h,
                          const mg_options *opt, void *stream, mg_batch **out) {
    set_error("");
    if (!out || n < 1 || !masks_dev || !dims || !h) {
        set_error("invalid batch arguments");
        return MG_ERR_ARG;
    }
    *out = nullptr;
    mg_batch *B = new (std::nothrow) mg_batch();
    if (!B) return MG_ERR_ALLOC;
    B->n = n;
    if (opt) B->opt = *opt;
    else mg_default_options(&B->opt);
    if (B->opt.precision != MG_FP64) {
        set_error("the batched solver runs in FP64");
        delete B;
        return MG_ERR_ARG;
    }
    if (kPersistentEnabled && (B->opt.n_pre + B->opt.n_post) % 2 != 0) {
        // the cycle programs keep the finest iterate in buffer 0 between cycles
        set_error("the batched solver needs an even number of finest-level passes per cycle");
        delete B;
        return MG_ERR_ARG;
    }
    B->stream = (hipStream_t)stream;
    mg_status st = MG_OK;
    try {
        if (!B->stream) {
            BHIP(hipStreamCreate(&B->stream));
            B->own_stream = true;
        }
        build_batch(B, masks_dev, dims, h);
        if (!kPersistentEnabled) {
            *out = B;
            return MG_OK;
        }
        // store program (needs the per-patch finest tile lists)
        Planner P{B, 2};
        P.cur.assign(n, std::vector<int>(MAXL, 0));
        P.begin(PH_STORE);
        for (int p = 0; p < n; p++)
            for (int t : P.tl(p, 0))
                if (t >= 0) P.items.push_back(BItem{p, 0, t, 0, Seg{}});
        P.end();
        B->store = finish(B, P);
        BHIP(hipStreamSynchronize(B->stream));
    } catch (const BFail &f) {
        st = f.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        st = MG_ERR_ALLOC;
    }
    if (st != MG_OK) {
        mg_destroy_batch(B);
        return st;
    }
    *out = B;
    return MG_OK;
}

mg_status mg_solve_batch(mg_batch *B, const double *const *rho_dev, double *const *phi_dev,
                         const double *const *dirichlet_dev, double tol, mg_solve_info *infos, double *ms_out) {
    if (!B || !rho_dev || !phi_dev || !(tol > 0)) {
        set_error("invalid batch solve arguments");
        return MG_ERR_ARG;
    }
    for (int p = 0; p < B->n; p++)
        if (!rho_dev[p] || !phi_dev[p]) {
            set_error("null rho or phi in batch");
            return MG_ERR_ARG;
        }
    try {
        return solve_batch(B, rho_dev, phi_dev, dirichlet_dev, tol, infos, ms_out);
    } catch (const BFail &f) {
        return f.st;
    } catch (...) {
        set_error("unexpected internal error");
        return MG_ERR_HIP;
    }
}

int32_t mg_batch_size(const mg_batch *B) { return B ? B->n : 0; }

int32_t mg_batch_grid(const mg_batch *B) { return B ? B->grid : 0; }

int32_t mg_batch_phases(const mg_batch *B, int32_t order) {
    if (!B || (order != 1 && order != 2)) return 0;
    return B->cycle[order].nph;
}

}  // extern "C"
