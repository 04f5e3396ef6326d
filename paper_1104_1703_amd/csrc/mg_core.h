// Internal declarations of the gfx950 masked multigrid library.
// Layout of every level: dense (nz, ny, nx) box, x fastest.  Work is issued
// only over "active tiles" (TX x TY x TZ blocks holding at least one active
// cell), so cost follows the active cell count, as the paper's hierarchy
// restricted to active cells does (Sec. 2, Fig. "hierarchy").
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <type_traits>
#include <vector>

#include "mg.h"

#include "tiles.h"

namespace mg {

constexpr int MAXL = 16;
constexpr int MAXS = 8;                    // levels handled by the one-workgroup kernel
constexpr size_t SMALL_MAX_CELLS = 4096;   // first level handled there has at most this many cells
constexpr int SMALL_LDS_MAX = 160 * 1024;  // LDS of one gfx950 workgroup

// Default planes per smoother work item of a level (a hierarchy may use other
// depths with kernel instances: 8, 16, 32 on the finest level, 2, 4, 8 on
// coarse levels; OrderData::depth holds the one in use).
constexpr int item_depth(int level) {
    return level == 0 ? SEG_TILES_FINE * TZ : level == 1 ? SEGZ_COARSE1 : SEGZ_COARSE;
}
constexpr bool depth_supported(int level, int depth) {
    return level == 0 ? (depth == 8 || depth == 16 || depth == 32) : (depth == 2 || depth == 4 || depth == 8);
}
// Coarse-level option value selecting 8^3 cube items for plain passes (the
// passes that apply the prolongation keep the default march).
constexpr int DEPTH_CUBE = 1;
// Calls f(std::integral_constant<int, D>()) with D the finest-level item depth
// in use (the kernel instance to launch).
template <typename F>
inline void with_fine_depth(int depth, F &&f) {
    if (depth == 8) f(std::integral_constant<int, 8>());
    else if (depth == 32) f(std::integral_constant<int, 32>());
    else f(std::integral_constant<int, 16>());
}

// Stop test of the solve loop evaluated on the device by the norm's final
// sum (the same FP64 comparisons as the host's): halt when sqrt(sum) <= thresh,
// when it is not finite, or (check_switch) when sqrt(sum) / rprev > eta.
struct StopTest {
    double thresh, rprev, eta;
    int check_switch, pad;
};

// Per boundary order data of one level (index 1 = first order, 2 = second).
struct OrderData {
    double *d = nullptr;   // operator diagonal (coarse levels), 0 off the active set
    float *d32 = nullptr;  // float copy for the mixed-precision inner cycle
    int *tiles = nullptr;  // active tile ids (device)
    Seg *segs = nullptr;   // smoother work items (device)
    unsigned long long *pmask = nullptr;  // per item and plane activity masks (device)
    unsigned long long *pmask2 = nullptr; // the same for fused pairs of passes (4-cell halo; fuse_passes)
    unsigned long long *pmask3 = nullptr; // finest level: masks with a 3-cell halo for the pass with the residual
    // level 1, FP64 pass with the prolongation on load: whole 8-plane tiles as
    // work items and their masks (that pass fits 4 blocks per CU, not 5, and
    // one round of tiles beats two rounds of 4-plane items)
    Seg *segs8 = nullptr;
    unsigned long long *pmask8 = nullptr;
    int nsegs8 = 0;
    int ntiles = 0, nsegs = 0;
    int depth = 0;  // planes per work item of segs (its masks hold depth + 4 words per item)
    bool cube = false;  // coarse levels: plain passes over 8^3 cubes loaded whole (no z march)
    int64_t nact = 0;
};

struct Level {
    int nx = 0, ny = 0, nz = 0;
    double h = 0;
    size_t n = 0;
    int ntx = 0, nty = 0, ntz = 0;
    int32_t *cnt = nullptr;   // active finest descendants per cell
    uint8_t *code = nullptr;  // level 0: diagonal of the cell equation (6..12), CODE_OFF (0) if inactive
    OrderData od[3];
    const int *halt = nullptr;          // the hierarchy's halt flag: cycle kernels exit when set
    double *x[2] = {nullptr, nullptr};  // ping-pong iterate
    double *f = nullptr;                // right-hand side
    float *x32[2] = {nullptr, nullptr};
    float *f32 = nullptr;
};

struct Graph {
    hipGraphExec_t exec = nullptr;
    int order = 0, parity = 0;
    bool mixed = false, decide = false;
};

}  // namespace mg

namespace mg {
constexpr int KT_MAX_LAUNCHES = 1024;  // launches one kernel-timing record holds
}

struct mg_hierarchy {
    mg_options opt;
    hipStream_t stream = nullptr;
    bool own_stream = false;        // created here because the caller passed the null stream
    int device = 0;
    int nlev_geom = 0;
    int nlev[3] = {0, 0, 0};
    int ls[3] = {-1, -1, -1};       // first level run by the one-workgroup kernel, per order (-1: none)
    mg::Level lev[mg::MAXL];
    int hold_left = 0;
    int coarse_order_state = 0;     // order whose tiles the coarse x buffers are clean for
    double *part = nullptr;         // per-block partial sums (device)
    int part_cap = 0;
    double *norm_dev = nullptr;     // finalised sums (device, 4 doubles)
    double *norm_host = nullptr;    // pinned mirror (coherent host memory, mapped)
    double *norm_map = nullptr;     // device address of norm_host
    int *halt_dev = nullptr;        // set by the device stop test; read by every cycle kernel
    mg::StopTest *stop_dev = nullptr;
    double *scratch = nullptr;      // finest-level float64 scratch (fold/residual of the fine level)
    double *scratch2 = nullptr;
    std::vector<void *> allocs;
    std::vector<mg::Graph> graphs;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t evq[2] = {nullptr, nullptr};  // ends of the (at most two) cycles in flight
    // input norms written by the device straight to norm_host: events
    // without a system-scope fence (the value does not pass through the
    // device caches)
    hipEvent_t evn[2] = {nullptr, nullptr};
    // optional timing of one kind of finest-level red-black launch inside
    // solves (kt_on: 0 off, 1 plain passes, 2 the pass with the residual, 3
    // the pass with the prolongation, 4 the pass forming the input norm): an
    // event pair per launch (the kernel's own start and end), up to
    // kt_ev.size() / 2 launches
    int kt_on = 0;
    std::vector<hipEvent_t> kt_ev;
    int kt_used = 0;
};

namespace mg {

// -------- the solve loop in phases (api.hip) --------
// State of one solve (Sec. 2 iteration with the Sec. 4 order switch) between
// its phases; see phase_begin.
struct SolveState {
    mg_solve_info *info = nullptr;
    double *phi = nullptr;
    double tol = 0.0;
    int order = 2;
    bool mixed = false;
    int parity = 0;
    int n = 0;  // cycles done
    double rprev = 0.0, rref = 0.0;
    mg_status st = MG_NOT_CONVERGED;
    bool active = false;  // another cycle is due
    int host_slot = 0;    // norm_host entry holding the last finished cycle's norm
};
// begin: enqueue fold and the two reference norms; start: read them (the
// caller has synchronised the hierarchy's stream); cycle_enqueue: one cycle
// with its norm copy; cycle_finish: stop test and order switch (stream
// synchronised); end: enqueue the store of phi and the end event.
mg_status phase_begin(mg_hierarchy *H, const double *rho, double *phi, const double *B, double tol,
                      mg_solve_info *info, SolveState &S);
// init: begin's host part alone (state, order, coarse buffers cleaned); the
// caller computes the fold and both reference norms itself and stores them
// in norm_host[0] (of the guess) and norm_host[1] (of f) before start.
mg_status phase_init(mg_hierarchy *H, double *phi, double tol, mg_solve_info *info, SolveState &S);
mg_status phase_start(mg_hierarchy *H, SolveState &S);
mg_status phase_cycle_enqueue(mg_hierarchy *H, SolveState &S);
mg_status phase_cycle_finish(mg_hierarchy *H, SolveState &S);
mg_status phase_end(mg_hierarchy *H, SolveState &S);

// -------- allocation / errors (api.hip) --------
void *dev_alloc(mg_hierarchy *H, size_t bytes);
void set_error(const std::string &s);
bool hip_ok(hipError_t e, const char *what);

// -------- setup kernels (setup.hip) --------
void launch_validate(const int8_t *mask, int nx, int ny, int nz, unsigned long long *bad, hipStream_t s);
void launch_count0(const int8_t *mask, int32_t *cnt, size_t n, hipStream_t s);
void launch_count_up(const Level &fine, const Level &coarse, hipStream_t s);
void launch_code0(const Level &L, unsigned long long *nact, hipStream_t s);
void launch_diag(const Level &L, int level, int order, double *d, unsigned long long *nact, hipStream_t s);
void launch_tile_flags(const Level &L, int level, int order, uint8_t *flags, hipStream_t s);
void launch_to_float(const double *a, float *b, size_t n, hipStream_t s);
// Activity masks of the smoother work items of `od` (npl planes per item)
// for an xy halo of 2 (single passes), 3 (the finest pass that also forms the
// residual) or 4 (fused pairs of passes) cells.
void launch_item_masks(const Level &L, int level, int order, const OrderData &od, int npl, unsigned long long *pm,
                       hipStream_t s, int halo = 2);

// -------- smoother (smooth.hip) --------
// One red-black pass over the segments of `od`; xin == nullptr reads zero.
// On the finest level, events e0 / e1 (if given) take the kernel's own start
// and end times (hipExtLaunchKernel); the launch status is returned.
hipError_t launch_rbgs(const Level &L, int level, const OrderData &od, const double *xin, double *xout,
                       const double *f, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_rbgs32(const Level &L, int level, const OrderData &od, const float *xin, float *xout,
                         const float *f, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// A pass over the 8^3 cubes of a coarse level (od.cube) that also forms the
// residual and its R1 restriction fc onto the next coarser level C (in
// order `order`): bit for bit launch_rbgs followed by launch_restrict.
void launch_rbgs_restrict(const Level &L, const Level &C, int order, const OrderData &od, const double *xin,
                          double *xout, const double *f, double *fc, hipStream_t s);
void launch_rbgs_restrict32(const Level &L, const Level &C, int order, const OrderData &od, const float *xin,
                            float *xout, const float *f, float *fc, hipStream_t s);
// A finest-level pass (od.pmask3 must exist; xin may be null) that also forms
// the residual of its result and its R1 restriction fc onto level 1 in order
// `order`: bit for bit launch_rbgs followed by launch_restrict.
hipError_t launch_rbgs_res_fine(const Level &L, const Level &C, int order, const OrderData &od, const double *xin,
                                double *xout, const double *f, double *fc, hipStream_t s, hipEvent_t e0 = nullptr,
                                hipEvent_t e1 = nullptr);
hipError_t launch_rbgs_res_fine32(const Level &L, const Level &C, int order, const OrderData &od, const float *xin,
                                  float *xout, const float *f, float *fc, hipStream_t s, hipEvent_t e0 = nullptr,
                                  hipEvent_t e1 = nullptr);
// A finest-level FP64 pass (xin != nullptr) that also writes the residual
// norm partials of its input xin, one per work item, to part[0 .. od.nsegs):
// the same values, bit for bit, as launch_resnorm's partials of xin.
hipError_t launch_rbgs_norm(const Level &L, const OrderData &od, const double *xin, double *xout, const double *f,
                            double *part, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// A pass that first adds the P2 prolongation of the coarse iterate xc (level
// level + 1, dims of C) to xin on active cells, as launch_prolong would, then
// relaxes; xin is left unchanged.
hipError_t launch_rbgs_prolong(const Level &L, int level, const OrderData &od, const Level &C, const double *xc,
                               const double *xin, double *xout, const double *f, hipStream_t s,
                               hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_rbgs_prolong32(const Level &L, int level, const OrderData &od, const Level &C, const float *xc,
                                 const float *xin, float *xout, const float *f, hipStream_t s,
                                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Two passes in one launch (fused; od.pmask2 must exist): the same result as
// two launch_rbgs calls xin -> tmp -> xout, bit for bit.
void launch_rbgs2(const Level &L, int level, const OrderData &od, const double *xin, double *xout, const double *f,
                  hipStream_t s);
void launch_rbgs2_32(const Level &L, int level, const OrderData &od, const float *xin, float *xout, const float *f,
                     hipStream_t s);
// The prolongation pass and the pass after it in one launch (finest level).
void launch_rbgs2_prolong(const Level &L, const OrderData &od, const Level &C, const double *xc, const double *xin,
                          double *xout, const double *f, hipStream_t s);
void launch_rbgs2_prolong32(const Level &L, const OrderData &od, const Level &C, const float *xc, const float *xin,
                            float *xout, const float *f, hipStream_t s);

// -------- small levels in one workgroup (coarse.hip) --------
size_t small_lds_bytes(const mg_hierarchy *H, int order, int ls, bool f32);
int small_init();  // usable dynamic LDS bytes of the one-workgroup kernel (0: none)
// One call MG(ls) for the levels ls..deepest; x0 is level ls's iterate (in/out).
void launch_small(const mg_hierarchy *H, int order, int ls, bool zero_start, const double *f0, double *x0,
                  hipStream_t s);
void launch_small32(const mg_hierarchy *H, int order, int ls, bool zero_start, const float *f0, float *x0,
                    hipStream_t s);

// -------- transfers and reductions (transfer.hip) --------
void launch_fold(const Level &L, const OrderData &od, const double *rho, const double *B, const double *phi,
                 double *f, double *x, hipStream_t s);
void launch_store(const Level &L, const OrderData &od, const double *x, double *phi, hipStream_t s);
void launch_copy_masked(const Level &L, int level, const OrderData &od, const double *src, double *dst,
                        hipStream_t s);
// Sum of squares of (L x - f) (or of f alone when x == nullptr) into part[],
// then a fixed-order total into out[slot]; with `stop` the total also runs
// the stop test and sets the level's halt flag.
void launch_resnorm(const Level &L, int level, const OrderData &od, const double *x, const double *f, double *part,
                    double *out, int slot, hipStream_t s, const StopTest *stop = nullptr,
                    double *host_out = nullptr);
// The fixed-order total of n partials into out[slot], with `stop` also the
// stop test on it (halt flag of L) -- the final step of launch_resnorm;
// host_out (device address of coherent host memory): the total is also
// stored there at system scope.
void launch_finalize(const Level &L, const double *part, int n, double *out, int slot, const StopTest *stop,
                     hipStream_t s, double *host_out = nullptr);
// Device flags of the solve loop (small kernels, safe inside captured graphs).
void launch_set_halt(int *halt, int v, hipStream_t s);
void launch_set_stop(StopTest *st, double thresh, double rprev, double eta, int check_switch, hipStream_t s);
void launch_residual(const Level &L, int level, const OrderData &od, const double *x, const double *f, double *r,
                     hipStream_t s);
void launch_restrict(const Level &L, const Level &C, int level, int order, const double *x, const double *f,
                     double *fc, hipStream_t s);
void launch_restrict32(const Level &L, const Level &C, int level, int order, const float *x, const float *f,
                       float *fc, hipStream_t s);
void launch_prolong(const Level &L, const Level &C, int level, int order, const double *xc, double *x,
                    hipStream_t s);
void launch_prolong32(const Level &L, const Level &C, int level, int order, const float *xc, float *x,
                      hipStream_t s);
void launch_zero_tiles(const Level &L, const OrderData &od, double *x, hipStream_t s);
void launch_zero_tiles32(const Level &L, const OrderData &od, float *x, hipStream_t s);
// Mixed precision: outer FP64 residual norm of the finest level that also
// writes r32 = f - L x in float (the inner right-hand side).
void launch_resnorm32(const Level &L, const OrderData &od, const double *x, const double *f, float *r32, double *part,
                      double *out, int slot, hipStream_t s);
// Mixed precision, end of an outer iteration: xo = x + e on active cells (xo
// must differ from x), then the FP64 residual norm of xo and r32 = f - L xo
// in float.
void launch_axpy_resnorm32(const Level &L, const OrderData &od, const double *x, const float *e, double *xo,
                           const double *f, float *r32, double *part, double *out, int slot, hipStream_t s,
                           const StopTest *stop = nullptr, double *host_out = nullptr);

}  // namespace mg
