// Batched solver: many independent masked grids (AMR-level patches of uneven
// size and depth) solved together.
//
// Every patch has its own hierarchy, operators, boundary-order switch and
// stop test, exactly as a single solve (Sec. 2-4).  One multigrid cycle of
// all unconverged patches runs as a short program of launches, each launch
// one phase of the cycle for every patch that reaches it: a red-black pass
// over the smoother items of level l, the residual with R1 restriction, the
// small levels (one 1024-thread workgroup per patch), the residual-norm
// partials and their per-patch fixed-order sums.  A block takes one work
// item, which names a patch level (a descriptor in device memory) and an
// item of that level's own lists, and runs the single-grid kernels' device
// code on it.  So each patch gets bit for bit what a single solve gives it,
// while one cycle of hundreds of patches costs as many launches as one cycle
// of one grid.  A state word per patch gates every item: the program of each
// boundary order serves the patches now in that order; converged patches
// skip.  The host reads all per-patch norms once per cycle and takes each
// patch's decisions with the single-grid solve loop's own code.
//
// A cycle's first finest pass runs ahead of those decisions, in a program of
// its own that serves every unconverged patch in either order (the finest
// level is the same in both): it reads the iterate from buffer 0, writes
// buffer 1 and forms the residual norm of its input, bit for bit the
// norm march's (patches solved whole in one workgroup or with one level get
// the march there instead).  After the one synchronisation a patch that
// stops keeps buffer 0; the others run the rest of the cycle in the order
// their decision gives.
//
// The programs keep the finest iterate in buffer 0 between cycles.  Options
// they do not cover (an odd number of finest-level passes per cycle, no
// post-smoothing, a zero-pass relaxation from a zero start) run each patch's
// own captured cycles in lockstep instead: one round enqueues one cycle per
// unconverged patch and synchronises once.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <new>

#include "coarse_core.h"
#include "march_core.h"

namespace mg {
namespace {

constexpr int FINE_Z = SEG_TILES_FINE * TZ;  // planes of a finest-level smoother item
constexpr int NTS = 1024;                     // threads of the small-level workgroup (as coarse.hip)
constexpr int WBITS = 24;                     // BRef::w: item index in the low bits, selector above
constexpr int IDX_MASK = (1 << WBITS) - 1;

// One level of one patch as the phases see it; one table per boundary order,
// entry patch * MAXL + level.
struct BLev {
    int nx, ny, nz, ntx, nty;
    int cnx, cny, cnz, cntx, cnty;  // next coarser level (0 if none)
    double h2, ih2;
    double *x[2];
    double *f;
    const uint8_t *code;                 // level 0 (else null)
    const double *d;                     // coarse levels: diagonal of this order (else null)
    const Seg *segs;                     // smoother items of this level and order
    const unsigned long long *pm;        // their activity masks
    const int *tiles;                    // active tiles
    double *cx[2];                       // next coarser level: iterate,
    double *cf;                          //   right-hand side,
    const double *cd;                    //   diagonal of this order,
    const int *ctiles;                   //   active tiles of this order
};

// Work item: descriptor index and (item index | selector << WBITS).  Selector
// bits: 1 = iterate buffer read, 2 = start from zero (no read), 4 = coarse
// iterate buffer of a prolongation pass.
struct BRef {
    int lev, w;
};

enum : int {
    K_SM0,    // red-black pass, finest level
    K_SM0P,   //   ... applying P2 from level 1 on load
    K_SM1,    // red-black pass, level 1
    K_SM1P,
    K_SM2,    // red-black pass, levels 2 and coarser
    K_SM2P,
    K_RES0,   // residual march of the finest level with R1 onto level 1
    K_RESC,   // residual and R1 from a coarse level, one coarse (tile, plane) per item
    K_SMALL,  // MG(ls) of one patch in one workgroup
    K_NORM,   // residual-norm partials of the finest level
    K_FIN,    // per-patch fixed-order sum of the partials
    K_FOLD,   // Dirichlet fold and guess load of the finest level
    K_STORE,  // finest iterate back to phi
    K_SM0N,   // red-black pass, finest level, with the residual-norm partials of its input
};

// Block -> work item; false for grid padding and for patches this program
// does not serve.
__device__ __forceinline__ bool take(const BRef *__restrict__ refs, int count, const int *__restrict__ state,
                                     int order, BRef &r) {
    const int w = rb::xcd_item(blockIdx.x, gridDim.x);
    if (w >= count) return false;
    r = refs[w];
    return state[r.lev / MAXL] == order;
}

// NORMIN: the pass also writes its item's partial of the residual norm of
// its input to part[poff + position] (the single-grid norm-forming pass).
template <bool FINE, int SEGZ, bool PRO, bool NORMIN = false>
__global__ __launch_bounds__(rb::NT, NORMIN ? 4 : 5) void kb_smooth(const BRef *__restrict__ refs, int count,
                                                       const BLev *__restrict__ lev, const int *__restrict__ state,
                                                       int order, double *__restrict__ part = nullptr, int poff = 0) {
    __shared__ rb::RbgsLds<double, FINE, PRO> lds;
    BRef r;
    if (!take(refs, count, state, order, r)) return;
    const BLev &L = lev[r.lev];
    const int idx = r.w & IDX_MASK, sel = r.w >> WBITS, a = sel & 1;
    const double sq = rb::rbgs_item<double, FINE, SEGZ, PRO, NORMIN>(
        lds, (sel & 2) ? nullptr : L.x[a], L.x[a ^ 1], L.f, L.code, L.d, L.nx, L.ny, L.nz, L.h2, L.segs[idx],
        L.pm + (size_t)idx * (SEGZ + 4), PRO ? L.cx[(sel >> 2) & 1] : nullptr, L.cnx, L.cny, L.cnz, L.ih2);
    if constexpr (NORMIN) {
        const double t = tr::block_sum(sq);
        if (threadIdx.x == 0) part[poff + rb::xcd_item(blockIdx.x, gridDim.x)] = t;
    }
}

template <int MODE>
__global__ __launch_bounds__(tr::NT) void kb_residual(const BRef *__restrict__ refs, int count,
                                                      const BLev *__restrict__ lev, const int *__restrict__ state,
                                                      int order, double *__restrict__ part, int poff = 0) {
    __shared__ tr::ResLds<double> lds;
    BRef r;
    if (!take(refs, count, state, order, r)) return;
    const BLev &L = lev[r.lev];
    const int idx = r.w & IDX_MASK, sel = r.w >> WBITS;
    constexpr bool RS = MODE == tr::RM_RESTRICT;
    const double sq = tr::residual_item<double, FINE_Z, MODE>(
        lds, (sel & 2) ? nullptr : L.x[sel & 1], L.f, L.code, L.nx, L.ny, L.nz, L.ih2, L.segs[idx],
        L.pm + (size_t)idx * (FINE_Z + 4), RS ? L.cd : nullptr, RS ? L.cnx : 0, RS ? L.cny : 0,
        RS ? L.cf : nullptr, nullptr, nullptr, nullptr);
    if constexpr (!RS) {
        const double t = tr::block_sum(sq);
        if (threadIdx.x == 0) part[poff + rb::xcd_item(blockIdx.x, gridDim.x)] = t;
    }
}

__global__ __launch_bounds__(tr::NT) void kb_restrict(const BRef *__restrict__ refs, int count,
                                                      const BLev *__restrict__ lev, const int *__restrict__ state,
                                                      int order) {
    BRef r;
    if (!take(refs, count, state, order, r)) return;
    const BLev &L = lev[r.lev];
    const int idx = r.w & IDX_MASK, sel = r.w >> WBITS;
    const tr::TileCoord t = tr::tile_cell(L.ctiles[idx / TZ], idx % TZ, L.cntx, L.cnty, L.cnx, L.cny, L.cnz);
    tr::restrict_cell<double, false>(t, L.cnx, L.cny, L.cd, L.nx, L.ny, L.nz, L.ih2, nullptr, L.d, L.x[sel & 1], L.f,
                                     L.cf);
}

__global__ __launch_bounds__(NTS) void kb_small(const BRef *__restrict__ refs, int count,
                                                const BLev *__restrict__ lev, const int *__restrict__ state,
                                                int order, const small::SmallLevels<double> *__restrict__ sl) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    if ((int)blockIdx.x >= count) return;
    const BRef r = refs[blockIdx.x];
    const int p = r.lev / MAXL;
    if (state[p] != order) return;
    const BLev &L = lev[r.lev];
    const int sel = r.w >> WBITS;
    small::small_tail<double, NTS>(reinterpret_cast<double *>(smem_raw), sl[p], L.f, L.x[sel & 1], (sel & 2) == 0);
}

// Per patch p: the sum of part[first[p] .. first[p] + cnt[p]) in the same
// order as the single-grid norm's final sum, into out[2 p + slot].
__global__ __launch_bounds__(1024) void kb_finalize(const int *__restrict__ first, const int *__restrict__ cnt,
                                                    int npatch, const double *__restrict__ part,
                                                    double *__restrict__ out, int slot, const int *__restrict__ state,
                                                    int order) {
    __shared__ double sm[1024];
    const int p = blockIdx.x;
    if (p >= npatch || state[p] != order) return;
    const double *pp = part + first[p];
    const int n = cnt[p];
    double v = 0.0;
    for (int q = threadIdx.x; q < n; q += 1024) v += pp[q];
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[2 * p + slot] = sm[0];
}

__global__ __launch_bounds__(tr::NT) void kb_fold(const BRef *__restrict__ refs, int count,
                                                  const BLev *__restrict__ lev, const int *__restrict__ state,
                                                  int order, const double *const *__restrict__ rho,
                                                  const double *const *__restrict__ dir,
                                                  const double *const *__restrict__ phi) {
    BRef r;
    if (!take(refs, count, state, order, r)) return;
    const BLev &L = lev[r.lev];
    const int p = r.lev / MAXL, idx = r.w & IDX_MASK;
    tr::fold_cell(tr::tile_cell(L.tiles[idx / TZ], idx % TZ, L.ntx, L.nty, L.nx, L.ny, L.nz), L.nx, L.ny, L.ih2,
                  L.code, rho[p], dir[p], phi[p], L.f, L.x[0]);
}

__global__ __launch_bounds__(tr::NT) void kb_store(const BRef *__restrict__ refs, int count,
                                                   const BLev *__restrict__ lev, const int *__restrict__ state,
                                                   int order, double *const *__restrict__ phi) {
    BRef r;
    if (!take(refs, count, state, order, r)) return;
    const BLev &L = lev[r.lev];
    const int p = r.lev / MAXL, idx = r.w & IDX_MASK, sel = r.w >> WBITS;
    tr::store_cell(tr::tile_cell(L.tiles[idx / TZ], idx % TZ, L.ntx, L.nty, L.nx, L.ny, L.nz), L.nx, L.ny, L.code,
                   L.x[sel & 1], phi[p]);
}

__host__ __device__ inline unsigned grid8(int items) { return (unsigned)(((items + 7) / 8) * 8); }

// One launch of a program.
struct Launch {
    int kind, first, count;
    size_t lds;    // dynamic LDS (K_SMALL)
    int slot;      // K_FIN: norm slot
    int poff = 0;  // K_NORM, K_SM0N: offset of the launch's partials
    int lay = 0;   // K_FIN: 0 = partials of every patch in patch order, 1 = the pre-cycle layout
};

// ------------------------------------------------------------ persistent
// The persistent engine runs whole programs in one cooperative launch: the
// launches of the per-phase engine become phases separated by a grid-wide
// barrier, and every block walks the phase's work items in the order the
// per-phase kernel's blocks take them (virtual block vb -> item
// xcd_item(vb, grid)), so each item runs the same device code on the same
// data and partial sums land in the same slots: results are bit for bit
// those of the per-phase engine.  Blocks are 256 threads with PERSIST_LDS
// of dynamic LDS (four blocks per CU).  The small-level call runs with 256
// threads (its sweeps are in place per colour and its transfers per cell,
// so the thread count does not change a result), its levels in LDS where
// they fit PERSIST_LDS, else in a global-memory area of the block's own
// (block barriers only).
constexpr int PERSIST_LDS = 38 * 1024;  // dynamic LDS of a block (with the static part, 4 per CU)
constexpr unsigned PERSIST_SPIN_LIMIT = 1u << 22;    // barrier polls (seconds in all), then err
static_assert(sizeof(rb::RbgsLds<double, true, true>) <= PERSIST_LDS &&
                  sizeof(rb::RbgsLds<double, false, true>) <= PERSIST_LDS &&
                  sizeof(tr::ResLds<double>) <= PERSIST_LDS && 1024 * sizeof(double) <= PERSIST_LDS,
              "every phase's LDS fits a persistent block");

struct PSeg {
    const Launch *k;    // device copy of a program's launches
    int nk;
    int order;
    const int *state;
};

struct PArgs {
    PSeg seg[3];
    int nseg;
    const BRef *refs;
    const BLev *lev[3];
    const small::SmallLevels<double> *sl[3];
    double *part, *norm2;
    const int *nfirst, *ncnt, *nfirst1, *ncnt1;
    int npatch;
    const double *const *rho;
    const double *const *dir;
    double *const *phi;
    unsigned *bar;  // [2]: arrivals, generation
    int *err;       // set when a barrier wait exceeds its bound
    const int *sbytes[3];  // per order and patch: bytes of its small-level call's levels
    double *gsmall;        // per block: gsmall_elems doubles for a call above PERSIST_LDS
    long long gsmall_elems;
};

// Grid-wide barrier of a co-resident launch.  One thread per block: an
// agent-scope release fence (the block's global writes, ordered before it by
// the block barrier, are written back from this XCD's L2), a relaxed arrival
// on the counter, a relaxed spin on the generation word, then one
// agent-scope acquire fence (this XCD's L2 and the CU's L1 are invalidated).
// The spin issues plain coherent loads: an acquire load per iteration would
// invalidate the XCD's L2 on every poll while other blocks still work.  The
// last arrival acquires every other block's release (it read their arrivals)
// and releases before it bumps the generation.  The wait is bounded: past
// the bound it raises err and goes on, so every wave reaches the kernel's
// end (the host then reports the error).
__device__ void persist_sync(unsigned *bar, int *err) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived =
            __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (arrived == gridDim.x) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > PERSIST_SPIN_LIMIT) {
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Work item of virtual block vb of a phase with `grid` virtual blocks, as
// the per-phase kernel's block vb takes it.
__device__ __forceinline__ bool ptake(const BRef *refs, const Launch &k, int vb, int grid, const int *state,
                                      int order, BRef &r, int &w) {
    w = rb::xcd_item(vb, grid);
    if (w >= k.count) return false;
    r = refs[k.first + w];
    return state[r.lev / MAXL] == order;
}

template <bool FINE, int SEGZ, bool PRO, bool NORMIN = false>
__device__ __attribute__((noinline)) void p_smooth(unsigned char *smem, const BRef r, int w, const BLev *lev, double *part, int poff) {
    auto &lds = *reinterpret_cast<rb::RbgsLds<double, FINE, PRO> *>(smem);
    const BLev &L = lev[r.lev];
    const int idx = r.w & IDX_MASK, sel = r.w >> WBITS, a = sel & 1;
    const double sq = rb::rbgs_item<double, FINE, SEGZ, PRO, NORMIN>(
        lds, (sel & 2) ? nullptr : L.x[a], L.x[a ^ 1], L.f, L.code, L.d, L.nx, L.ny, L.nz, L.h2, L.segs[idx],
        L.pm + (size_t)idx * (SEGZ + 4), PRO ? L.cx[(sel >> 2) & 1] : nullptr, L.cnx, L.cny, L.cnz, L.ih2);
    if constexpr (NORMIN) {
        const double t = tr::block_sum(sq);
        if (threadIdx.x == 0) part[poff + w] = t;
    }
}

template <int MODE>
__device__ __attribute__((noinline)) void p_residual(unsigned char *smem, const BRef r, int w, const BLev *lev, double *part, int poff) {
    auto &lds = *reinterpret_cast<tr::ResLds<double> *>(smem);
    const BLev &L = lev[r.lev];
    const int idx = r.w & IDX_MASK, sel = r.w >> WBITS;
    constexpr bool RS = MODE == tr::RM_RESTRICT;
    const double sq = tr::residual_item<double, FINE_Z, MODE>(
        lds, (sel & 2) ? nullptr : L.x[sel & 1], L.f, L.code, L.nx, L.ny, L.nz, L.ih2, L.segs[idx],
        L.pm + (size_t)idx * (FINE_Z + 4), RS ? L.cd : nullptr, RS ? L.cnx : 0, RS ? L.cny : 0,
        RS ? L.cf : nullptr, nullptr, nullptr, nullptr);
    if constexpr (!RS) {
        const double t = tr::block_sum(sq);
        if (threadIdx.x == 0) part[poff + w] = t;
    }
}

__device__ __attribute__((noinline)) void p_small(unsigned char *smem, const small::SmallLevels<double> &S,
                                                  const double *f0, double *x0, bool load_x) {
    small::small_tail<double, rb::NT>(reinterpret_cast<double *>(smem), S, f0, x0, load_x);
}

__device__ __attribute__((noinline)) void p_small_global(double *area, const small::SmallLevels<double> &S,
                                                         const double *f0, double *x0, bool load_x) {
    small::small_tail<double, rb::NT, false>(area, S, f0, x0, load_x);
}

__device__ __attribute__((noinline)) void p_cell(int kind, const BLev &L, int idx, int sel, const double *rho,
                                                 const double *dir, double *phi) {
    switch (kind) {
        case K_RESC: {
            const tr::TileCoord t = tr::tile_cell(L.ctiles[idx / TZ], idx % TZ, L.cntx, L.cnty, L.cnx, L.cny, L.cnz);
            tr::restrict_cell<double, false>(t, L.cnx, L.cny, L.cd, L.nx, L.ny, L.nz, L.ih2, nullptr, L.d,
                                             L.x[sel & 1], L.f, L.cf);
            break;
        }
        case K_FOLD:
            tr::fold_cell(tr::tile_cell(L.tiles[idx / TZ], idx % TZ, L.ntx, L.nty, L.nx, L.ny, L.nz), L.nx, L.ny,
                          L.ih2, L.code, rho, dir, phi, L.f, L.x[0]);
            break;
        case K_STORE:
            tr::store_cell(tr::tile_cell(L.tiles[idx / TZ], idx % TZ, L.ntx, L.nty, L.nx, L.ny, L.nz), L.nx, L.ny,
                           L.code, L.x[sel & 1], phi);
            break;
        default: break;
    }
}

__global__ __launch_bounds__(rb::NT, 4) void kb_persist(PArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    bool first = true;
    for (int si = 0; si < A.nseg; si++) {
        const PSeg S = A.seg[si];
        const int order = S.order;
        const BLev *lev = A.lev[order];
        for (int i = 0; i < S.nk; i++) {
            if (!first) persist_sync(A.bar, A.err);
            first = false;
            const Launch k = S.k[i];
            if (k.kind == K_FIN) {
                // per patch: the per-phase kernel's 1024-lane fixed-order sum, four lanes per thread
                const int *fi = k.lay ? A.nfirst1 : A.nfirst;
                const int *cn = k.lay ? A.ncnt1 : A.ncnt;
                double *sm = reinterpret_cast<double *>(smem);
                for (int p = blockIdx.x; p < A.npatch; p += gridDim.x) {
                    if (S.state[p] != order) continue;
                    const double *pp = A.part + fi[p];
                    const int n = cn[p];
                    for (int lane = threadIdx.x; lane < 1024; lane += rb::NT) {
                        double v = 0.0;
                        for (int q = lane; q < n; q += 1024) v += pp[q];
                        sm[lane] = v;
                    }
                    __syncthreads();
                    for (int o = 512; o > 0; o >>= 1) {
                        for (int lane = threadIdx.x; lane < o; lane += rb::NT) sm[lane] += sm[lane + o];
                        __syncthreads();
                    }
                    if (threadIdx.x == 0) A.norm2[2 * p + k.slot] = sm[0];
                    __syncthreads();
                }
                continue;
            }
            if (k.kind == K_SMALL) {
                for (int vb = blockIdx.x; vb < k.count; vb += gridDim.x) {
                    const BRef r = A.refs[k.first + vb];
                    const int p = r.lev / MAXL;
                    if (S.state[p] != order) continue;
                    const BLev &L = lev[r.lev];
                    const int sel = r.w >> WBITS;
                    if (A.sbytes[order][p] <= PERSIST_LDS)
                        p_small(smem, A.sl[order][p], L.f, L.x[sel & 1], (sel & 2) == 0);
                    else
                        p_small_global(A.gsmall + (size_t)blockIdx.x * A.gsmall_elems, A.sl[order][p], L.f,
                                       L.x[sel & 1], (sel & 2) == 0);
                    __syncthreads();
                }
                continue;
            }
            const int grid = (int)grid8(k.count);
            for (int vb = blockIdx.x; vb < grid; vb += gridDim.x) {
                BRef r;
                int w;
                if (!ptake(A.refs, k, vb, grid, S.state, order, r, w)) continue;
                const BLev &L = lev[r.lev];
                const int idx = r.w & IDX_MASK, sel = r.w >> WBITS, p = r.lev / MAXL;
                switch (k.kind) {
                    case K_SM0: p_smooth<true, FINE_Z, false>(smem, r, w, lev, nullptr, 0); break;
                    case K_SM0P: p_smooth<true, FINE_Z, true>(smem, r, w, lev, nullptr, 0); break;
                    case K_SM1: p_smooth<false, SEGZ_COARSE1, false>(smem, r, w, lev, nullptr, 0); break;
                    case K_SM1P: p_smooth<false, SEGZ_COARSE1, true>(smem, r, w, lev, nullptr, 0); break;
                    case K_SM2: p_smooth<false, SEGZ_COARSE, false>(smem, r, w, lev, nullptr, 0); break;
                    case K_SM2P: p_smooth<false, SEGZ_COARSE, true>(smem, r, w, lev, nullptr, 0); break;
                    case K_SM0N: p_smooth<true, FINE_Z, false, true>(smem, r, w, lev, A.part, k.poff); break;
                    case K_RES0: p_residual<tr::RM_RESTRICT>(smem, r, w, lev, nullptr, 0); break;
                    case K_NORM: p_residual<tr::RM_NORM>(smem, r, w, lev, A.part, k.poff); break;
                    case K_RESC:
                    case K_FOLD:
                    case K_STORE: p_cell(k.kind, L, idx, sel, A.rho[p], A.dir[p], A.phi[p]); break;
                    default: break;
                }
                __syncthreads();  // the next item reuses the block's LDS
            }
        }
    }
}

__global__ void kb_zero_bar(unsigned *bar, int *err) {
    if (threadIdx.x < 2) bar[threadIdx.x] = 0u;
    if (threadIdx.x == 0) *err = 0;
}

}  // namespace
}  // namespace mg

// ------------------------------------------------------------------ host --

struct mg_batch {
    int n = 0;
    mg_options opt;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<mg_hierarchy *> patches;  // all enqueue on `stream`
    std::vector<void *> allocs;           // batch-owned device memory
    bool phased_ok = false;               // phase programs built
    bool use_phases = true;
    // phase programs: begin (fold, reference norms), pre (the next cycle's
    // first finest pass with the norm of its input), the rest of one cycle per
    // order, end (store)
    struct Prog {
        std::vector<mg::Launch> k;
        hipGraphExec_t exec = nullptr;
    };
    Prog begin, end, pre, cycle[3];
    mg::BRef *refs = nullptr;                    // device, all programs' work items
    mg::BLev *lev[3] = {};                       // device [n * MAXL] per order
    mg::small::SmallLevels<double> *sl[3] = {};  // device [n] per order
    int *state[4] = {};                          // device [n]: [0] every patch 2, [o] this cycle's order-o patches,
                                                 //   [3] the patches of the pre program
    int *pin_state = nullptr;                    // pinned [3n]
    int *nfirst = nullptr, *ncnt = nullptr;      // device [n]: each patch's norm partials within a norm phase
    int *nfirst1 = nullptr, *ncnt1 = nullptr;    // ... within the pre program
    double *part = nullptr;
    double *norm2 = nullptr;       // device [2n]
    double *norm2_host = nullptr;  // pinned
    const double **in_rho = nullptr, **in_dir = nullptr;  // device [n] each
    double **in_phi = nullptr;
    const double **pin_ptrs = nullptr;  // pinned [3n]: rho, dirichlet, phi
    int small_lim = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // persistent engine: device copies of the programs' launches (begin,
    // end, pre, cycle 1, cycle 2), the block's LDS, the grid barrier, the
    // co-resident grid size
    bool persist_ok = false;
    bool use_persist = false;
    mg::Launch *dk[5] = {};
    int plds = 0;  // dynamic LDS of a persistent block
    const int *psbytes[3] = {nullptr, nullptr, nullptr};  // per order, per patch: small-level call bytes
    double *gsmall = nullptr;     // per persistent block: a global area for the larger small-level calls
    long long gsmall_elems = 0;
    unsigned *pbar = nullptr;
    int *perr = nullptr;
    int *perr_host = nullptr;  // pinned
    int pgrid = 0;
    // host copies of the tables the programs read, for their validation
    std::vector<mg::BRef> refs_host;
    std::vector<int> nfirst_h, ncnt_h, nfirst1_h, ncnt1_h;
    int part_cap = 0;
};

namespace mg {
namespace {

struct BFail {
    mg_status st;
};
struct Unsupported {};

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

// Emits the phase programs.  cur[p][l]: buffer holding patch p's level-l
// iterate, tracked as the single-grid cycle does.
struct Planner {
    mg_batch *B;
    int o;
    std::vector<Launch> *out;
    std::vector<BRef> &refs;
    std::vector<std::array<int, MAXL>> cur;
    std::vector<char> skip;  // patches whose first finest pass of a cycle runs in the pre program

    Planner(mg_batch *b, int order, std::vector<BRef> &r) : B(b), o(order), out(nullptr), refs(r) {
        cur.assign(b->n, std::array<int, MAXL>{});
    }
    static int pack(int idx, int sel) {
        if (idx < 0 || idx > IDX_MASK) throw Unsupported{};
        return idx | (sel << WBITS);
    }
    const OrderData &od(int p, int l) const { return B->patches[p]->lev[l].od[l == 0 ? 2 : o]; }
    void open(int kind, size_t lds = 0, int slot = 0) {
        out->push_back(Launch{kind, (int)refs.size(), 0, lds, slot});
    }
    void close() {
        Launch &k = out->back();
        k.count = (int)refs.size() - k.first;
        if (k.count == 0) out->pop_back();
    }
    void add(int p, int l, int n, int sel) {
        for (int i = 0; i < n; i++) refs.push_back(BRef{p * MAXL + l, pack(i, sel)});
    }
    // one red-black pass on level l (pro: the first post pass, with P2 on load)
    void pass(const std::vector<int> &ps, int l, bool zero, bool pro) {
        open((l == 0 ? K_SM0 : l == 1 ? K_SM1 : K_SM2) + (pro ? 1 : 0));
        for (int p : ps)
            add(p, l, od(p, l).nsegs, cur[p][l] | (zero ? 2 : 0) | (pro ? cur[p][l + 1] << 2 : 0));
        close();
        for (int p : ps) cur[p][l] ^= 1;
    }
    void smooth(const std::vector<int> &ps, int l, int passes, bool zero) {
        if (ps.empty()) return;
        if (passes == 0) {
            if (zero) throw Unsupported{};  // the single-grid cycle zeroes the tiles here
            return;
        }
        for (int j = 0; j < passes; j++) pass(ps, l, zero && j == 0, false);
    }
    // MG(l) for the patches ps, in the single-grid cycle's order of steps
    void mg(const std::vector<int> &ps, int l, bool zero) {
        const mg_options &op = B->opt;
        std::vector<int> sm, last, reg;
        for (int p : ps) {
            const mg_hierarchy *H = B->patches[p];
            if (l == H->ls[o]) sm.push_back(p);
            else if (l == H->nlev[o] - 1) last.push_back(p);
            else reg.push_back(p);
        }
        if (!sm.empty()) {
            size_t lds = 0;
            for (int p : sm) lds = std::max(lds, small_lds_bytes(B->patches[p], o, l, false));
            if (lds > (size_t)B->small_lim) throw Unsupported{};
            open(K_SMALL, lds);
            for (int p : sm) add(p, l, 1, cur[p][l] | (zero ? 2 : 0));
            close();
        }
        smooth(last, l, op.n_coarse_sweeps, zero);
        if (reg.empty()) return;
        if (l == 0 && !skip.empty()) {
            // the pre program ran the first pass of the patches marked in skip
            std::vector<int> extra;
            for (int p : reg)
                if (!skip[p]) extra.push_back(p);
            smooth(extra, 0, 1, zero);
            smooth(reg, 0, op.n_pre - 1, zero);
        } else {
            smooth(reg, l, op.n_pre, zero);
        }
        open(l == 0 ? K_RES0 : K_RESC);
        for (int p : reg) {
            const Level &C = B->patches[p]->lev[l + 1];
            if (C.od[o].ntiles) add(p, l, l == 0 ? od(p, 0).nsegs : C.od[o].ntiles * TZ, cur[p][l]);
        }
        close();
        for (int c = 0; c < op.n_cycles; c++) mg(reg, l + 1, c == 0);
        if (op.n_post == 0) throw Unsupported{};  // the single-grid cycle prolongs without a pass
        pass(reg, l, false, true);
        smooth(reg, l, op.n_post - 1, false);
    }
    // residual-norm partials of every patch's finest level and their sums into slot
    void norm(bool with_x, int slot) {
        open(K_NORM);
        for (int p = 0; p < B->n; p++) add(p, 0, od(p, 0).nsegs, with_x ? cur[p][0] : 2);
        close();
        out->push_back(Launch{K_FIN, 0, B->n, 0, slot});
    }
    // pre program: the first finest pass of the next cycle, which also forms
    // the norm partials of the current iterate (patches marked in skip), the
    // residual-norm march of the others, and every patch's sum into slot 0;
    // first/cnt: each patch's partials in this layout
    void pre(std::vector<int> &first, std::vector<int> &cnt) {
        int at = 0;
        open(K_SM0N);
        for (int p = 0; p < B->n; p++)
            if (skip[p]) {
                first[p] = at;
                cnt[p] = od(p, 0).nsegs;
                at += cnt[p];
                add(p, 0, cnt[p], 0);
            }
        close();
        open(K_NORM);
        out->back().poff = at;
        int bt = 0;
        for (int p = 0; p < B->n; p++)
            if (!skip[p]) {
                first[p] = at + bt;
                cnt[p] = od(p, 0).nsegs;
                bt += cnt[p];
                add(p, 0, cnt[p], 0);
            }
        close();
        Launch fin{K_FIN, 0, B->n, 0, 0};
        fin.lay = 1;
        out->push_back(fin);
    }
    void tiles0(int kind) {
        open(kind);
        for (int p = 0; p < B->n; p++) add(p, 0, od(p, 0).ntiles * TZ, 0);
        close();
    }
};

// Level descriptors of one order.
std::vector<BLev> descriptors(mg_batch *B, int o) {
    std::vector<BLev> t((size_t)B->n * MAXL);
    memset(t.data(), 0, t.size() * sizeof(BLev));
    for (int p = 0; p < B->n; p++) {
        const mg_hierarchy *H = B->patches[p];
        for (int l = 0; l < H->nlev[o]; l++) {
            const Level &L = H->lev[l];
            const OrderData &d = L.od[l == 0 ? 2 : o];
            BLev &e = t[(size_t)p * MAXL + l];
            e.nx = L.nx; e.ny = L.ny; e.nz = L.nz; e.ntx = L.ntx; e.nty = L.nty;
            e.h2 = L.h * L.h;
            e.ih2 = 1.0 / (L.h * L.h);
            e.x[0] = L.x[0]; e.x[1] = L.x[1]; e.f = L.f;
            e.code = l == 0 ? L.code : nullptr;
            e.d = l == 0 ? nullptr : L.od[o].d;
            e.segs = d.segs; e.pm = d.pmask; e.tiles = d.tiles;
            if (l + 1 < H->nlev[o]) {
                const Level &C = H->lev[l + 1];
                e.cnx = C.nx; e.cny = C.ny; e.cnz = C.nz; e.cntx = C.ntx; e.cnty = C.nty;
                e.cx[0] = C.x[0]; e.cx[1] = C.x[1]; e.cf = C.f;
                e.cd = C.od[o].d;
                e.ctiles = C.od[o].tiles;
            }
        }
    }
    return t;
}

// Small-level descriptors of one order (as the single-grid launch builds them).
std::vector<small::SmallLevels<double>> small_levels(mg_batch *B, int o) {
    std::vector<small::SmallLevels<double>> sl(B->n);
    for (int p = 0; p < B->n; p++) {
        small::SmallLevels<double> &S = sl[p];
        memset(&S, 0, sizeof(S));
        const mg_hierarchy *H = B->patches[p];
        const int ls = H->ls[o];
        if (ls < 0) continue;
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
    return sl;
}

// Host-side check of every table the phase kernels read, before any of them
// runs: each work item's patch, level, item index and selector against the
// patch hierarchy it refers to (the level exists in the program's order and
// holds the buffers the kernel dereferences; the item index is below that
// level's item or tile count; the level's items have the depth the kernel
// instance marches, so its masks lie inside the mask array), each launch's
// item range inside the item table, each norm partial offset inside the
// partial buffer, and each small-level launch's LDS at least what its
// patches' levels need.  Returns the number of violations (the first few
// are written to *msg).
int validate_tables(const mg_batch *B, std::string *msg) {
    int bad = 0;
    auto fail = [&](const std::string &s) {
        if (bad++ < 8 && msg) *msg += s + "; ";
    };
    const int n = B->n;
    const int nref = (int)B->refs_host.size();
    struct ProgRef {
        const mg_batch::Prog *g;
        int order;
        const char *name;
    };
    const ProgRef progs[] = {{&B->begin, 2, "begin"}, {&B->end, 2, "end"}, {&B->pre, 2, "pre"},
                             {&B->cycle[1], 1, "cycle1"}, {&B->cycle[2], 2, "cycle2"}};
    for (const ProgRef &pr : progs) {
        const int o = pr.order;
        for (const Launch &k : pr.g->k) {
            const std::string where = std::string(pr.name) + " kind " + std::to_string(k.kind);
            if (k.kind == K_FIN) {
                const std::vector<int> &fi = k.lay ? B->nfirst1_h : B->nfirst_h;
                const std::vector<int> &cn = k.lay ? B->ncnt1_h : B->ncnt_h;
                if (k.count != n || (int)fi.size() != n || (int)cn.size() != n) fail(where + ": patch count");
                else
                    for (int p = 0; p < n; p++)
                        if (fi[p] < 0 || cn[p] < 0 || fi[p] + cn[p] > B->part_cap) fail(where + ": partial range");
                continue;
            }
            if (k.first < 0 || k.count < 0 || k.first + k.count > nref) {
                fail(where + ": item range outside the table");
                continue;
            }
            if ((k.kind == K_NORM || k.kind == K_SM0N) && (k.poff < 0 || k.poff + k.count > B->part_cap))
                fail(where + ": partials outside the buffer");
            for (int i = k.first; i < k.first + k.count; i++) {
                const BRef r = B->refs_host[i];
                const int p = r.lev / MAXL, l = r.lev % MAXL, idx = r.w & IDX_MASK, sel = r.w >> WBITS;
                if (r.lev < 0 || p >= n) {
                    fail(where + ": patch out of range");
                    continue;
                }
                const mg_hierarchy *H = B->patches[p];
                if (l >= H->nlev[o] || sel < 0 || sel > 7) {
                    fail(where + ": level or selector out of range");
                    continue;
                }
                const Level &L = H->lev[l];
                const OrderData &od = L.od[l == 0 ? 2 : o];
                const bool bufs = L.x[0] && L.x[1] && L.f;
                const bool has_c = l + 1 < H->nlev[o];
                switch (k.kind) {
                    case K_SM0:
                    case K_SM0P:
                    case K_SM0N:
                    case K_SM1:
                    case K_SM1P:
                    case K_SM2:
                    case K_SM2P: {
                        const int want_l = (k.kind == K_SM1 || k.kind == K_SM1P) ? 1 : (k.kind == K_SM2 || k.kind == K_SM2P) ? 2 : 0;
                        const int depth = want_l == 0 ? FINE_Z : want_l == 1 ? SEGZ_COARSE1 : SEGZ_COARSE;
                        const bool pro = k.kind == K_SM0P || k.kind == K_SM1P || k.kind == K_SM2P;
                        if ((want_l < 2 ? l != want_l : l < 2) || idx >= od.nsegs || od.depth != depth || !bufs ||
                            !od.segs || !od.pmask || (l == 0 ? !L.code : !od.d))
                            fail(where + ": smoother item");
                        if (pro && (!has_c || !H->lev[l + 1].x[(sel >> 2) & 1])) fail(where + ": prolongation source");
                        break;
                    }
                    case K_RES0:
                        if (l != 0 || idx >= od.nsegs || od.depth != FINE_Z || !has_c || !bufs || !L.code ||
                            !H->lev[1].f || !H->lev[1].od[o].d)
                            fail(where + ": finest residual item");
                        break;
                    case K_RESC:
                        if (l < 1 || !has_c || !bufs || !od.d || idx >= H->lev[l + 1].od[o].ntiles * TZ ||
                            !H->lev[l + 1].od[o].tiles || !H->lev[l + 1].f)
                            fail(where + ": coarse restriction item");
                        break;
                    case K_SMALL:
                        if (l != H->ls[o] || !bufs || k.lds < small_lds_bytes(H, o, l, false) ||
                            k.lds > (size_t)B->small_lim)
                            fail(where + ": small-level item");
                        break;
                    case K_NORM:
                        if (l != 0 || idx >= od.nsegs || od.depth != FINE_Z || !L.f || !L.code)
                            fail(where + ": norm item");
                        break;
                    case K_FOLD:
                    case K_STORE:
                        if (l != 0 || idx >= od.ntiles * TZ || !od.tiles || !bufs) fail(where + ": tile-plane item");
                        break;
                    default:
                        fail(where + ": unknown kind");
                }
            }
        }
    }
    return bad;
}

// Builds the phase programs; false (and the lockstep engine) when the
// options or a patch need a step the programs do not have.
bool build_programs(mg_batch *B) {
    const int n = B->n;
    std::vector<BRef> refs;
    // patches whose finest level takes passes in both orders: the first of a
    // cycle's passes runs in the pre program, which also forms the norm of
    // the cycle's input; the others get the residual-norm march there
    std::vector<char> skip(n, 0);
    for (int p = 0; p < n; p++) {
        const mg_hierarchy *H = B->patches[p];
        skip[p] = B->opt.n_pre >= 1 && H->ls[1] != 0 && H->ls[2] != 0 && H->nlev[1] > 1 && H->nlev[2] > 1;
    }
    std::vector<int> first1(n), cnt1(n);
    try {
        for (int o = 1; o <= 2; o++) {
            Planner P(B, o, refs);
            P.out = &B->cycle[o].k;
            P.skip = skip;
            std::vector<int> all(n);
            for (int p = 0; p < n; p++) {
                all[p] = p;
                P.cur[p][0] = skip[p] ? 1 : 0;
            }
            P.mg(all, 0, false);
            for (int p = 0; p < n; p++)
                if (P.cur[p][0] != 0) throw Unsupported{};  // odd number of finest-level passes
        }
        {
            Planner P(B, 2, refs);
            P.out = &B->pre.k;
            P.skip = skip;
            P.pre(first1, cnt1);
        }
        Planner P(B, 2, refs);
        P.out = &B->begin.k;
        P.tiles0(K_FOLD);
        P.norm(false, 1);
        P.norm(true, 0);
        P.out = &B->end.k;
        P.tiles0(K_STORE);
    } catch (const Unsupported &) {
        for (auto *g : {&B->begin, &B->end, &B->pre, &B->cycle[1], &B->cycle[2]}) g->k.clear();
        return false;
    }
    // each patch's partials within a norm phase (every norm phase lists all
    // patches' finest items in patch order)
    std::vector<int> first(n), cnt(n);
    int part_cap = 1, acc = 0;
    for (int p = 0; p < n; p++) {
        first[p] = acc;
        cnt[p] = B->patches[p]->lev[0].od[2].nsegs;
        acc += cnt[p];
    }
    part_cap = std::max(part_cap, acc);
    B->refs_host = refs;
    B->nfirst_h = first;
    B->ncnt_h = cnt;
    B->nfirst1_h = first1;
    B->ncnt1_h = cnt1;
    B->part_cap = part_cap;
    {
        std::string why;
        if (validate_tables(B, &why) != 0) {
            set_error("batch tables failed validation: " + why);
            throw BFail{MG_ERR_HIP};
        }
    }
    B->refs = upload(B, refs);
    B->nfirst = upload(B, first);
    B->ncnt = upload(B, cnt);
    B->nfirst1 = upload(B, first1);
    B->ncnt1 = upload(B, cnt1);
    B->part = balloc<double>(B, (size_t)part_cap);
    for (int o = 1; o <= 2; o++) {
        B->lev[o] = upload(B, descriptors(B, o));
        B->sl[o] = upload(B, small_levels(B, o));
    }
    B->lev[0] = B->lev[2];
    for (int s = 0; s < 4; s++) B->state[s] = balloc<int>(B, n);
    std::vector<int> all2(n, 2);
    BHIP(hipMemcpyAsync(B->state[0], all2.data(), n * sizeof(int), hipMemcpyHostToDevice, B->stream));
    BHIP(hipStreamSynchronize(B->stream));
    B->in_rho = (const double **)balloc<double *>(B, n);
    B->in_dir = (const double **)balloc<double *>(B, n);
    B->in_phi = balloc<double *>(B, n);
    BHIP(hipHostMalloc((void **)&B->pin_ptrs, 3 * (size_t)n * sizeof(double *), hipHostMallocDefault));
    BHIP(hipHostMalloc((void **)&B->pin_state, 3 * (size_t)n * sizeof(int), hipHostMallocDefault));
    return true;
}

// Device copies of the programs for the persistent engine and its
// co-resident grid; false when the device cannot run it.
bool build_persistent(mg_batch *B) {
    int dev = 0, ncu = 0, coop = 0, per = 0;
    BHIP(hipGetDevice(&dev));
    BHIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) {
        (void)hipGetLastError();
        return false;
    }
    // per order and patch, the bytes of its small-level call's levels; the
    // largest sizes the global area of a block (calls above PERSIST_LDS)
    size_t gmax = 0;
    for (int o = 1; o <= 2; o++) {
        std::vector<int> sb(B->n, 0);
        for (int p = 0; p < B->n; p++) {
            const mg_hierarchy *H = B->patches[p];
            if (H->ls[o] >= 0) sb[p] = (int)small_lds_bytes(H, o, H->ls[o], false);
            if (sb[p] > PERSIST_LDS) gmax = std::max(gmax, (size_t)sb[p]);
        }
        B->psbytes[o] = upload(B, sb);
    }
    B->psbytes[0] = B->psbytes[2];
    B->plds = PERSIST_LDS;
    BHIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)kb_persist, rb::NT, PERSIST_LDS));
    B->pgrid = (per * ncu) / 8 * 8;
    if (B->pgrid < 8) return false;
    B->gsmall_elems = (long long)((gmax / sizeof(double) + 31) / 32 * 32);
    if (B->gsmall_elems > 0) B->gsmall = balloc<double>(B, (size_t)B->pgrid * (size_t)B->gsmall_elems);
    const mg_batch::Prog *progs[5] = {&B->begin, &B->end, &B->pre, &B->cycle[1], &B->cycle[2]};
    for (int i = 0; i < 5; i++) B->dk[i] = upload(B, progs[i]->k);
    B->pbar = balloc<unsigned>(B, 2);
    B->perr = balloc<int>(B, 1);
    BHIP(hipHostMalloc((void **)&B->perr_host, sizeof(int), hipHostMallocDefault));
    return true;
}

void build_batch(mg_batch *B, const int8_t *const *masks, const int32_t *dims, const double *h) {
    const int n = B->n;
    BHIP(hipEventCreate(&B->ev0));
    BHIP(hipEventCreate(&B->ev1));
    B->patches.resize(n, nullptr);
    for (int p = 0; p < n; p++) {
        mg_options o = B->opt;
        o.use_graph = 1;  // the lockstep engine replays each patch's captured cycle
        // the phase kernels are instances for the default work-item depths
        o.tune = 0;
        o.item_depth_fine = o.item_depth_l1 = o.item_depth_coarse = 0;
        mg_hierarchy *H = nullptr;
        const mg_status st =
            mg_create_hierarchy(masks[p], dims[3 * p], dims[3 * p + 1], dims[3 * p + 2], h[p], &o, B->stream, &H);
        if (st != MG_OK) throw BFail{st};
        B->patches[p] = H;
    }
    B->norm2 = balloc<double>(B, 2 * (size_t)n);
    BHIP(hipHostMalloc((void **)&B->norm2_host, 2 * (size_t)n * sizeof(double), hipHostMallocDefault));
    // the small-level workgroup gets the LDS the patches' small levels were sized for
    B->small_lim = small_init();
    bool lds_ok = B->small_lim > 0;
    if (lds_ok && B->small_lim > 64 * 1024 - 1024 &&
        hipFuncSetAttribute((const void *)kb_small, hipFuncAttributeMaxDynamicSharedMemorySize, B->small_lim) !=
            hipSuccess) {
        (void)hipGetLastError();
        lds_ok = false;
    }
    B->phased_ok = lds_ok && build_programs(B);
    B->use_phases = B->phased_ok;
    B->persist_ok = B->phased_ok && build_persistent(B);
    BHIP(hipStreamSynchronize(B->stream));
}

void launch(mg_batch *B, const Launch &k, int order, const int *state) {
    const BRef *r = B->refs + k.first;
    const BLev *lev = B->lev[order];
    hipStream_t s = B->stream;
    const unsigned g = grid8(k.count);
    constexpr int NT = rb::NT;
    switch (k.kind) {
        case K_SM0: kb_smooth<true, FINE_Z, false><<<g, NT, 0, s>>>(r, k.count, lev, state, order); break;
        case K_SM0P: kb_smooth<true, FINE_Z, true><<<g, NT, 0, s>>>(r, k.count, lev, state, order); break;
        case K_SM1: kb_smooth<false, SEGZ_COARSE1, false><<<g, NT, 0, s>>>(r, k.count, lev, state, order); break;
        case K_SM1P: kb_smooth<false, SEGZ_COARSE1, true><<<g, NT, 0, s>>>(r, k.count, lev, state, order); break;
        case K_SM2: kb_smooth<false, SEGZ_COARSE, false><<<g, NT, 0, s>>>(r, k.count, lev, state, order); break;
        case K_SM2P: kb_smooth<false, SEGZ_COARSE, true><<<g, NT, 0, s>>>(r, k.count, lev, state, order); break;
        case K_RES0:
            kb_residual<tr::RM_RESTRICT><<<g, NT, 0, s>>>(r, k.count, lev, state, order, nullptr);
            break;
        case K_RESC: kb_restrict<<<g, NT, 0, s>>>(r, k.count, lev, state, order); break;
        case K_SMALL: kb_small<<<k.count, NTS, k.lds, s>>>(r, k.count, lev, state, order, B->sl[order]); break;
        case K_NORM:
            kb_residual<tr::RM_NORM><<<g, NT, 0, s>>>(r, k.count, lev, state, order, B->part, k.poff);
            break;
        case K_SM0N:
            kb_smooth<true, FINE_Z, false, true><<<g, NT, 0, s>>>(r, k.count, lev, state, order, B->part, k.poff);
            break;
        case K_FIN:
            kb_finalize<<<B->n, 1024, 0, s>>>(k.lay ? B->nfirst1 : B->nfirst, k.lay ? B->ncnt1 : B->ncnt, B->n,
                                              B->part, B->norm2, k.slot, state, order);
            break;
        case K_FOLD:
            kb_fold<<<g, NT, 0, s>>>(r, k.count, lev, state, order, B->in_rho, B->in_dir,
                                     (const double *const *)B->in_phi);
            break;
        case K_STORE: kb_store<<<g, NT, 0, s>>>(r, k.count, lev, state, order, B->in_phi); break;
        default: break;
    }
}

// One program on the batch stream, replayed from its captured graph when
// the options ask for graphs.
void run_program(mg_batch *B, mg_batch::Prog &g, int order, const int *state) {
    if (!B->opt.use_graph) {
        for (const Launch &k : g.k) launch(B, k, order, state);
        BHIP(hipGetLastError());
        return;
    }
    if (!g.exec) {
        hipGraph_t graph = nullptr;
        BHIP(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
        for (const Launch &k : g.k) launch(B, k, order, state);
        const hipError_t le = hipGetLastError();
        BHIP(hipStreamEndCapture(B->stream, &graph));
        BHIP(le);
        const hipError_t ie = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        BHIP(ie);
    }
    BHIP(hipGraphLaunch(g.exec, B->stream));
}

// Programs run back to back in one cooperative launch (a grid barrier
// between consecutive phases).  prog: 0 begin, 1 end, 2 pre, 3 cycle 1,
// 4 cycle 2.
struct PRun {
    int prog, order;
    const int *state;
};

void run_persist(mg_batch *B, std::initializer_list<PRun> runs) {
    const mg_batch::Prog *progs[5] = {&B->begin, &B->end, &B->pre, &B->cycle[1], &B->cycle[2]};
    PArgs A;
    memset(&A, 0, sizeof(A));
    for (const PRun &r : runs) {
        if (progs[r.prog]->k.empty()) continue;
        PSeg &s = A.seg[A.nseg++];
        s.k = B->dk[r.prog];
        s.nk = (int)progs[r.prog]->k.size();
        s.order = r.order;
        s.state = r.state;
    }
    if (A.nseg == 0) return;
    A.refs = B->refs;
    for (int o = 0; o < 3; o++) A.lev[o] = B->lev[o];
    for (int o = 1; o <= 2; o++) A.sl[o] = B->sl[o];
    A.sl[0] = A.sl[2];
    A.part = B->part;
    A.norm2 = B->norm2;
    A.nfirst = B->nfirst;
    A.ncnt = B->ncnt;
    A.nfirst1 = B->nfirst1;
    A.ncnt1 = B->ncnt1;
    A.npatch = B->n;
    A.rho = B->in_rho;
    A.dir = B->in_dir;
    A.phi = B->in_phi;
    A.bar = B->pbar;
    A.err = B->perr;
    for (int o = 0; o < 3; o++) A.sbytes[o] = B->psbytes[o];
    A.gsmall = B->gsmall;
    A.gsmall_elems = B->gsmall_elems;
    kb_zero_bar<<<1, 64, 0, B->stream>>>(B->pbar, B->perr);
    void *args[] = {&A};
    BHIP(hipLaunchCooperativeKernel((const void *)kb_persist, dim3(B->pgrid), dim3(rb::NT), args, (size_t)B->plds,
                                    B->stream));
}

// Waits for the batch stream (the norms were queued for copy) and checks
// the persistent launches' barrier flag.
void persist_wait(mg_batch *B) {
    BHIP(hipMemcpyAsync(B->perr_host, B->perr, sizeof(int), hipMemcpyDeviceToHost, B->stream));
    BHIP(hipStreamSynchronize(B->stream));
    if (*B->perr_host) {
        set_error("persistent batch launch: a grid barrier wait exceeded its bound");
        throw BFail{MG_ERR_HIP};
    }
}

mg_status first_error(const std::vector<SolveState> &S);
mg_status finish_batch(mg_batch *B, std::vector<SolveState> &S, mg_solve_info *infos, double *ms_out);

// The persistent engine: the steps of the per-phase engine, each program
// run as phases of one cooperative launch; per V-cycle one launch runs the
// cycle in each boundary order in use and then the next cycle's first
// finest pass with the norm of its input, followed by one copy of all
// per-patch norms and one synchronisation.
mg_status solve_batch_persistent(mg_batch *B, const double *const *rho, double *const *phi,
                                 const double *const *dir, double tol, mg_solve_info *infos, double *ms_out) {
    const int n = B->n;
    hipStream_t s = B->stream;
    std::vector<SolveState> S(n);
    BHIP(hipStreamSynchronize(s));  // no copy of an earlier solve still reads the staging
    BHIP(hipEventRecord(B->ev0, s));
    for (int p = 0; p < n; p++) {
        const mg_status st = phase_init(B->patches[p], phi[p], tol, &infos[p], S[p]);
        if (st != MG_OK) return st;
    }
    const double **pr = B->pin_ptrs, **pd = B->pin_ptrs + n, **pp = B->pin_ptrs + 2 * n;
    for (int p = 0; p < n; p++) {
        pr[p] = rho[p];
        pd[p] = dir ? dir[p] : nullptr;
        pp[p] = phi[p];
    }
    BHIP(hipMemcpyAsync((void *)B->in_rho, pr, n * sizeof(double *), hipMemcpyHostToDevice, s));
    BHIP(hipMemcpyAsync((void *)B->in_dir, pd, n * sizeof(double *), hipMemcpyHostToDevice, s));
    BHIP(hipMemcpyAsync((void *)B->in_phi, pp, n * sizeof(double *), hipMemcpyHostToDevice, s));
    run_persist(B, {{0, 2, B->state[0]}});
    BHIP(hipMemcpyAsync(B->norm2_host, B->norm2, 2 * n * sizeof(double), hipMemcpyDeviceToHost, s));
    persist_wait(B);
    for (int p = 0; p < n; p++) {
        mg_hierarchy *H = B->patches[p];
        H->norm_host[0] = B->norm2_host[2 * p];
        H->norm_host[1] = B->norm2_host[2 * p + 1];
        const mg_status st = phase_start(H, S[p]);
        if (st != MG_OK) return st;
    }
    // the first cycle's first finest pass with the norm of the initial iterate
    int *sp = B->pin_state;  // slot 0 of the pinned staging: the pre program's patches
    bool any = false;
    for (int p = 0; p < n; p++) {
        sp[p] = S[p].active ? 2 : 0;
        any |= S[p].active;
    }
    if (any) {
        BHIP(hipMemcpyAsync(B->state[3], sp, n * sizeof(int), hipMemcpyHostToDevice, s));
        run_persist(B, {{2, 2, B->state[3]}});
        BHIP(hipMemcpyAsync(B->norm2_host, B->norm2, 2 * n * sizeof(double), hipMemcpyDeviceToHost, s));
        persist_wait(B);
    }
    std::vector<int> run;
    while (true) {
        run.clear();
        for (int p = 0; p < n; p++)
            if (S[p].active) run.push_back(p);
        if (run.empty()) break;
        // the rest of this cycle in each order, then the next cycle's first
        // pass (forming this cycle's norm) for the same patches
        bool use[3] = {false, false, false};
        for (int o = 1; o <= 2; o++) {
            int *sv = B->pin_state + o * n;  // the previous round's copies have finished
            for (int p = 0; p < n; p++) {
                sv[p] = (S[p].active && S[p].order == o) ? o : 0;
                use[o] |= sv[p] != 0;
            }
            if (use[o]) BHIP(hipMemcpyAsync(B->state[o], sv, n * sizeof(int), hipMemcpyHostToDevice, s));
        }
        for (int p = 0; p < n; p++) sp[p] = S[p].active ? 2 : 0;
        BHIP(hipMemcpyAsync(B->state[3], sp, n * sizeof(int), hipMemcpyHostToDevice, s));
        if (use[2] && use[1])
            run_persist(B, {{4, 2, B->state[2]}, {3, 1, B->state[1]}, {2, 2, B->state[3]}});
        else if (use[2])
            run_persist(B, {{4, 2, B->state[2]}, {2, 2, B->state[3]}});
        else
            run_persist(B, {{3, 1, B->state[1]}, {2, 2, B->state[3]}});
        BHIP(hipMemcpyAsync(B->norm2_host, B->norm2, 2 * n * sizeof(double), hipMemcpyDeviceToHost, s));
        persist_wait(B);
        for (int p : run) {
            mg_hierarchy *H = B->patches[p];
            H->norm_host[0] = B->norm2_host[2 * p];
            S[p].host_slot = 0;
            S[p].parity = 0;  // the finished cycle's iterate is in buffer 0
            const mg_status st = phase_cycle_finish(H, S[p]);
            if (st != MG_OK) return st;
        }
    }
    run_persist(B, {{1, 2, B->state[0]}});
    persist_wait(B);
    return finish_batch(B, S, infos, ms_out);
}

mg_status first_error(const std::vector<SolveState> &S) {
    mg_status worst = MG_OK;
    for (const SolveState &s : S)
        if (s.st < 0 || (s.st == MG_NOT_CONVERGED && worst == MG_OK)) worst = s.st;
    return worst;
}

mg_status finish_batch(mg_batch *B, std::vector<SolveState> &S, mg_solve_info *infos, double *ms_out) {
    BHIP(hipEventRecord(B->ev1, B->stream));
    BHIP(hipEventSynchronize(B->ev1));
    float ms = 0.f;
    BHIP(hipEventElapsedTime(&ms, B->ev0, B->ev1));
    if (ms_out) *ms_out = ms;
    for (int p = 0; p < B->n; p++) {
        infos[p].status = S[p].st;
        infos[p].ms = ms;
    }
    return first_error(S);
}

// The phase engine: per cycle, one program launch per boundary order in
// use, one copy of all per-patch norms and one synchronisation.
mg_status solve_batch_phased(mg_batch *B, const double *const *rho, double *const *phi, const double *const *dir,
                             double tol, mg_solve_info *infos, double *ms_out) {
    const int n = B->n;
    hipStream_t s = B->stream;
    std::vector<SolveState> S(n);
    BHIP(hipStreamSynchronize(s));  // no copy of an earlier solve still reads the staging
    BHIP(hipEventRecord(B->ev0, s));
    for (int p = 0; p < n; p++) {
        const mg_status st = phase_init(B->patches[p], phi[p], tol, &infos[p], S[p]);
        if (st != MG_OK) return st;
    }
    const double **pr = B->pin_ptrs, **pd = B->pin_ptrs + n, **pp = B->pin_ptrs + 2 * n;
    for (int p = 0; p < n; p++) {
        pr[p] = rho[p];
        pd[p] = dir ? dir[p] : nullptr;
        pp[p] = phi[p];
    }
    BHIP(hipMemcpyAsync((void *)B->in_rho, pr, n * sizeof(double *), hipMemcpyHostToDevice, s));
    BHIP(hipMemcpyAsync((void *)B->in_dir, pd, n * sizeof(double *), hipMemcpyHostToDevice, s));
    BHIP(hipMemcpyAsync((void *)B->in_phi, pp, n * sizeof(double *), hipMemcpyHostToDevice, s));
    run_program(B, B->begin, 2, B->state[0]);
    BHIP(hipMemcpyAsync(B->norm2_host, B->norm2, 2 * n * sizeof(double), hipMemcpyDeviceToHost, s));
    BHIP(hipStreamSynchronize(s));
    for (int p = 0; p < n; p++) {
        mg_hierarchy *H = B->patches[p];
        H->norm_host[0] = B->norm2_host[2 * p];
        H->norm_host[1] = B->norm2_host[2 * p + 1];
        const mg_status st = phase_start(H, S[p]);
        if (st != MG_OK) return st;
    }
    // Every round: the pre program (the first finest pass of the next cycle,
    // which also forms the residual norm of the current iterate; it reads
    // buffer 0 and writes buffer 1, and the finest level is the same in both
    // orders), one synchronisation, each patch's stop test and order switch
    // on that norm, then the rest of the cycle for the patches that go on.  A
    // patch that stops keeps its iterate in buffer 0.  The first round's norm
    // is the initial one, already taken.
    std::vector<int> run;
    for (int round = 0;; round++) {
        run.clear();
        for (int p = 0; p < n; p++)
            if (S[p].active) run.push_back(p);
        if (run.empty()) break;
        int *sp = B->pin_state;  // slot 0 of the pinned staging: the pre program's patches
        for (int p = 0; p < n; p++) sp[p] = S[p].active ? 2 : 0;
        BHIP(hipMemcpyAsync(B->state[3], sp, n * sizeof(int), hipMemcpyHostToDevice, s));
        run_program(B, B->pre, 2, B->state[3]);
        BHIP(hipMemcpyAsync(B->norm2_host, B->norm2, 2 * n * sizeof(double), hipMemcpyDeviceToHost, s));
        BHIP(hipStreamSynchronize(s));
        if (round > 0) {
            for (int p : run) {
                mg_hierarchy *H = B->patches[p];
                H->norm_host[0] = B->norm2_host[2 * p];
                S[p].host_slot = 0;
                S[p].parity = 0;  // the finished cycle's iterate is in buffer 0
                const mg_status st = phase_cycle_finish(H, S[p]);
                if (st != MG_OK) return st;
            }
        }
        for (int o = 2; o >= 1; o--) {
            int *sv = B->pin_state + o * n;  // the previous round's copies have finished
            bool use = false;
            for (int p = 0; p < n; p++) {
                sv[p] = (S[p].active && S[p].order == o) ? o : 0;
                use |= sv[p] != 0;
            }
            if (!use) continue;
            BHIP(hipMemcpyAsync(B->state[o], sv, n * sizeof(int), hipMemcpyHostToDevice, s));
            run_program(B, B->cycle[o], o, B->state[o]);
        }
    }
    run_program(B, B->end, 2, B->state[0]);
    return finish_batch(B, S, infos, ms_out);
}

// The lockstep engine: every round enqueues one captured cycle (with its
// 8-byte norm copy) of each unconverged patch, then synchronises once and
// applies each patch's stop test and order switch (Sec. 2, Sec. 4).
mg_status solve_batch_lockstep(mg_batch *B, const double *const *rho, double *const *phi, const double *const *dir,
                               double tol, mg_solve_info *infos, double *ms_out) {
    const int n = B->n;
    std::vector<SolveState> S(n);
    BHIP(hipEventRecord(B->ev0, B->stream));
    for (int p = 0; p < n; p++) {
        const mg_status st = phase_begin(B->patches[p], rho[p], phi[p], dir ? dir[p] : nullptr, tol, &infos[p], S[p]);
        if (st != MG_OK) return st;
    }
    BHIP(hipStreamSynchronize(B->stream));
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
        BHIP(hipStreamSynchronize(B->stream));
        for (int p : run) {
            const mg_status st = phase_cycle_finish(B->patches[p], S[p]);
            if (st != MG_OK) return st;
        }
    }
    for (int p = 0; p < n; p++) {
        const mg_status st = phase_end(B->patches[p], S[p]);
        if (st != MG_OK) return st;
    }
    return finish_batch(B, S, infos, ms_out);
}

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" {

void mg_destroy_batch(mg_batch *B) {
    if (!B) return;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    for (auto *g : {&B->begin, &B->end, &B->pre, &B->cycle[1], &B->cycle[2]})
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
    for (mg_hierarchy *H : B->patches) mg_destroy_hierarchy(H);
    for (void *p : B->allocs) {
        if (B->opt.allocator.free) B->opt.allocator.free(p, B->opt.allocator.ctx);
        else if (!B->opt.allocator.alloc) (void)hipFree(p);
    }
    if (B->norm2_host) (void)hipHostFree(B->norm2_host);
    if (B->pin_ptrs) (void)hipHostFree((void *)B->pin_ptrs);
    if (B->pin_state) (void)hipHostFree(B->pin_state);
    if (B->perr_host) (void)hipHostFree(B->perr_host);
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
    if (B->opt.tune || B->opt.item_depth_fine || B->opt.item_depth_l1 || B->opt.item_depth_coarse) {
        set_error("the batched solver runs the default work-item depths (no tuning)");
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
    std::vector<mg_solve_info> tmp;
    try {
        if (!infos) {
            tmp.resize(B->n);
            infos = tmp.data();
        }
        if (B->use_phases && B->use_persist)
            return solve_batch_persistent(B, rho_dev, phi_dev, dirichlet_dev, tol, infos, ms_out);
        if (B->use_phases) return solve_batch_phased(B, rho_dev, phi_dev, dirichlet_dev, tol, infos, ms_out);
        return solve_batch_lockstep(B, rho_dev, phi_dev, dirichlet_dev, tol, infos, ms_out);
    } catch (const BFail &f) {
        return f.st;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return MG_ERR_ALLOC;
    } catch (...) {
        set_error("unexpected internal error");
        return MG_ERR_HIP;
    }
}

mg_status mg_batch_set_engine(mg_batch *B, int32_t phased) {
    if (!B) {
        set_error("null batch");
        return MG_ERR_ARG;
    }
    if (phased < 0 || phased > 2 || (phased && !B->phased_ok)) {
        set_error("the phase programs do not cover these options; the batch runs per patch");
        return MG_ERR_ARG;
    }
    if (phased == 2 && !B->persist_ok) {
        set_error("this device cannot run the persistent batch engine");
        return MG_ERR_ARG;
    }
    B->use_phases = phased != 0;
    B->use_persist = phased == 2;
    return MG_OK;
}

int32_t mg_batch_size(const mg_batch *B) { return B ? B->n : 0; }

int32_t mg_batch_grid(const mg_batch *B) {
    if (!B || !B->phased_ok) return 0;
    int m = 0;
    for (int o = 1; o <= 2; o++)
        for (const mg::Launch &k : B->cycle[o].k) m = std::max(m, k.count);
    for (const mg::Launch &k : B->pre.k) m = std::max(m, k.count);
    return m;
}

int32_t mg_batch_validate(const mg_batch *B, char *msg, int32_t len) {
    if (!B) return -1;
    std::string why;
    const int bad = B->phased_ok ? mg::validate_tables(B, &why) : 0;
    if (msg && len > 0) {
        strncpy(msg, why.c_str(), (size_t)len - 1);
        msg[len - 1] = 0;
    }
    return bad;
}

int32_t mg_batch_phases(const mg_batch *B, int32_t order) {
    if (!B || !B->phased_ok || (order != 1 && order != 2)) return 0;
    return (int32_t)(B->pre.k.size() + B->cycle[order].k.size());
}

}  // extern "C"
