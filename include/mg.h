/*
 * mg.h -- C ABI of the MI355X (gfx950) masked multigrid Poisson solver.
 *
 * Method: Guillet & Teyssier, "A Simple Multigrid Scheme for Solving the
 * Poisson Equation with Arbitrary Domain Boundaries" (arXiv:1104.1703).
 * The solver computes Phi with  Delta Phi = rho  on the cells where the
 * caller's mask is +1 (Eq. "poisson"), with Dirichlet values on the faces
 * between active and inactive cells (Sec. 2, Fig. "grid").
 *
 * Conventions for every entry point:
 *   - Fields are C-contiguous (nz, ny, nx) boxes, x fastest; linear index
 *     (k*ny + j)*nx + i.  Coarse level l has dims (n >> l) per axis and
 *     spacing h * 2^l.
 *   - Pointers named *_dev are DEVICE pointers on the current HIP device;
 *     the caller owns them and keeps them alive for the call.  Pointers
 *     named *_host or *out are host pointers.
 *   - `stream` is a hipStream_t passed as void*.  All device work of a
 *     hierarchy is enqueued on the stream given at creation; 0 makes the
 *     library create its own blocking stream (the legacy null stream cannot
 *     be captured into a graph).  Calls that return host values synchronise
 *     that stream.
 *   - Errors are reported as mg_status; nothing throws or aborts.  The text
 *     of the last error of the calling thread is mg_last_error().
 *   - A hierarchy is not re-entrant: one call at a time per hierarchy.
 */
#ifndef MG_H
#define MG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MG_OK = 0,
    MG_NOT_CONVERGED = 1,   /* max_cycles reached; phi holds the last iterate */
    MG_ERR_ARG = -1,        /* invalid argument (see each entry point) */
    MG_ERR_NO_ACTIVE = -2,  /* the mask has no active cell */
    MG_ERR_HIP = -3,        /* a HIP runtime call failed; see mg_last_error() */
    MG_ERR_DIVERGED = -4,   /* residual norm became non-finite */
    MG_ERR_ALLOC = -5       /* device allocation failed */
} mg_status;

typedef enum { MG_FP64 = 0, MG_MIXED = 1 } mg_precision;

/* Coarse-level boundary reconstruction (Sec. 3 second order, Sec. 4 first
 * order); AUTO starts in second order and switches at run time (Sec. 4). */
typedef enum { MG_BC_AUTO = 0, MG_BC_FIRST = 1, MG_BC_SECOND = 2 } mg_bc_order;

/* Optional device allocator (e.g. a framework's caching allocator).  When
 * alloc is NULL the library uses hipMalloc/hipFree. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx);
    void (*free)(void *ptr, void *ctx);
    void *ctx;
} mg_allocator;

typedef struct {
    int32_t n_pre;            /* smoothing passes before restriction (Sec. 2: 2) */
    int32_t n_post;           /* smoothing passes after prolongation (Sec. 2: 2) */
    int32_t n_cycles;         /* coarse iterations per level: 1 = V, 2 = W (Sec. 5.3) */
    int32_t n_coarse_sweeps;  /* passes on the deepest level (default 32) */
    int32_t min_coarse_dim;   /* stop coarsening below this edge (default 4) */
    int32_t max_cycles;       /* solve-loop cap (default 200) */
    int32_t precision;        /* mg_precision (default MG_FP64) */
    int32_t bc_order;         /* mg_bc_order (default MG_BC_AUTO) */
    double eta;               /* switch threshold on ||r_n+1||/||r_n|| (Sec. 4: 0.5) */
    int32_t first_order_hold; /* solves kept in first order after a switch (Sec. 4: 10) */
    int32_t use_graph;        /* 1 = replay each cycle as a captured hipGraph; 0 (default) =
                                 launch its kernels directly (measured faster for one solve) */
    int32_t fuse_passes;      /* 1 = run each pair of consecutive red-black passes on a level
                                 as one launch (two passes per march: x, f and the diagonal
                                 read once for both); same results bit for bit (default 0) */
    int32_t tune;             /* 1 = pick the planes per smoother work item of every level and
                                 boundary order by timing the compiled variants at creation
                                 (cached in the file named by MG_TUNE_CACHE, if set); 0 = the
                                 defaults below (default 0).  Every choice gives the same
                                 iterates bit for bit; only the order in which the residual
                                 norm's partial sums are added depends on it. */
    int32_t item_depth_fine;  /* planes per finest-level work item: 8, 16 or 32; 0 = default
                                 (16) or tuned.  A non-zero value is used as given. */
    int32_t item_depth_l1;    /* level 1: 2, 4 or 8; 0 = default (4) or tuned; 1 = plain passes
                                 over 8 x 8 x 8 cubes loaded whole (no z march; not with
                                 fuse_passes), the prolongation pass keeping the default */
    int32_t item_depth_coarse;/* levels >= 2: as item_depth_l1 (default 2) */
    int32_t fuse_restrict;    /* 1 (default) = the last finest-level pre-smoothing pass also forms
                                 the residual and its R1 restriction (3-cell halo; no separate
                                 residual pass); 0 = a residual pass after it.  Same results bit
                                 for bit; not with fuse_passes, which keeps the residual pass. */
    mg_allocator allocator;
} mg_options;

typedef struct {
    int32_t cycles;            /* iterations performed */
    int32_t order_used;        /* 1 or 2: boundary order at the end of the solve */
    int32_t switched_at_cycle; /* cycle after which AUTO switched, -1 if none */
    int32_t status;            /* same value as returned */
    double r_ref;              /* ||r(phi = 0)||_2 = ||f||_2 over active cells */
    double r0;                 /* residual norm of the initial guess */
    double r_final;            /* residual norm at return */
    double ms;                 /* wall time of the call on the stream (HIP events) */
    double history[257];       /* history[n] = ||r|| after cycle n, n <= 256 */
} mg_solve_info;

typedef struct mg_hierarchy mg_hierarchy; /* opaque */

/* Fill *o with the defaults listed above. */
void mg_default_options(mg_options *o);

/*
 * Build the multigrid hierarchy for a mask (Sec. 2 Fig. "hierarchy"; Sec. 3
 * mask colouring and recursive R1 averaging; Sec. 4 first-order sets).
 *   mask_dev : int8 device array (nz, ny, nx), +1 active, -1 inactive.  Only
 *              read during the call; the caller may free it afterwards.
 *   h        : cell width (> 0).  opt: NULL = defaults.  out: receives the
 *              handle, to be released with mg_destroy_hierarchy.
 * Errors: MG_ERR_ARG for NULL pointers, non-positive dims or h, a box of
 * 2^34 cells or more or a z-plane of 2^28 cells or more, mask values other
 * than +-1, or a non-inactive outermost cell layer; MG_ERR_NO_ACTIVE
 * when no cell is +1; MG_ERR_ALLOC / MG_ERR_HIP.
 */
mg_status mg_create_hierarchy(const int8_t *mask_dev, int32_t nx, int32_t ny, int32_t nz, double h,
                              const mg_options *opt, void *stream, mg_hierarchy **out);

/* Release all device memory of the hierarchy (NULL is a no-op). */
void mg_destroy_hierarchy(mg_hierarchy *H);

/*
 * Solve Delta phi = rho with Dirichlet values (Sec. 2 iteration repeated
 * until ||r||_2 <= tol * ||r(phi = 0)||_2; Sec. 4 runtime order switch).
 *   rho_dev       : float64 (nz, ny, nx), read on active cells.
 *   phi_dev       : float64 (nz, ny, nx): initial guess in, solution out on
 *                   active cells; inactive cells are not written.
 *   dirichlet_dev : float64 cell-centred field B or NULL (= 0).  The value on
 *                   the face between active i and inactive j is (B_i+B_j)/2.
 *   tol           : > 0.   info: NULL or receives the solve record.
 * Returns MG_OK, MG_NOT_CONVERGED, MG_ERR_DIVERGED, MG_ERR_ARG, MG_ERR_HIP.
 */
mg_status mg_solve(mg_hierarchy *H, const double *rho_dev, double *phi_dev, const double *dirichlet_dev, double tol,
                   mg_solve_info *info);

/* ||Delta phi - rho||_2 over active cells (Sec. 2 step 2) into *norm_out (host). */
mg_status mg_residual_norm(mg_hierarchy *H, const double *rho_dev, const double *phi_dev,
                           const double *dirichlet_dev, double *norm_out);

/* For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, tight serving loops): mg_residual_norm with its partial
 * sums in a static per-device scratch array of the library (1 MiB, held by
 * each device the library runs on until the process ends) instead of the
 * hierarchy's buffer.  Calls no allocator and does not synchronise: the norm
 * is written to norm_dev (device, one double) on the hierarchy's stream.
 * The calling thread's current device must be the hierarchy's (MG_ERR_ARG
 * otherwise).  MG_ERR_ARG when the finest level has more than 131008 work
 * items (a 32 x 8 x 16 cell column each; a full 512^3 box has 32768).  Like
 * mg_residual_norm it overwrites the hierarchy's finest right-hand side and
 * iterate.  All calls on one device share the scratch array: calls that
 * overlap on one device (on different streams or from several threads)
 * race; calls ordered on one stream do not. */
mg_status mg_residual_norm_noalloc(mg_hierarchy *H, const double *rho_dev, const double *phi_dev,
                                   const double *dirichlet_dev, double *norm_dev);

/* Static text of a status code. */
const char *mg_status_string(mg_status s);

/* Text of the last error raised on the calling thread ("" if none). */
const char *mg_last_error(void);

/* ---------------- introspection ---------------- */

/* Levels used by boundary order `order` (1 or 2; 0 = levels that exist
 * geometrically).  The deepest used level is the deepest non-empty one. */
int32_t mg_num_levels(const mg_hierarchy *H, int32_t order);

/* dims_out[0..2] = (nx, ny, nz) of level l. */
mg_status mg_level_dims(const mg_hierarchy *H, int32_t level, int32_t *dims_out);

/* Number of active cells of level l under boundary order `order`. */
int64_t mg_level_active(const mg_hierarchy *H, int32_t level, int32_t order);

/* Planes per smoother work item of level l in boundary order `order` (the
 * default, the option's or the tuned value; work items are 32 x 8 cell
 * columns), 1 when its plain passes run over whole 8 x 8 x 8 cubes; -1 for
 * an invalid level or order.  Levels run by the
 * one-workgroup small-level kernel keep their lists but use none. */
int32_t mg_level_item_depth(const mg_hierarchy *H, int32_t level, int32_t order);

/* Copy the integer mask counts of level l (active finest descendants per
 * cell, int32, dims of level l) into a device array (Sec. 3 R1 of the mask). */
mg_status mg_level_counts(const mg_hierarchy *H, int32_t level, int32_t *counts_dev);

/* Copy the operator diagonal d (the cell's coefficient in h^2 * Laplacian,
 * negated; 0 on inactive cells) of level l and order into a float64 device
 * array.  Level 0: 6 active-neighbour faces + 2 per boundary face (Sec. 3,
 * boundary on the face); coarse levels: active neighbours + 1/theta. */
mg_status mg_level_diag(const mg_hierarchy *H, int32_t level, int32_t order, double *d_dev);

/* ---------------- single steps (Sec. 2 iteration), FP64 ---------------- */
/* All fields below are float64 device boxes of the named level.  Inputs are
 * read on active cells only; outputs are written on every cell (0 off the
 * active set unless stated). */

/* Right-hand side with the Dirichlet values folded in: f = rho - (1/h^2)
 * sum over boundary faces of (B_i + B_j); the finest system is then
 * (1/h^2)(sum_active x_j - d_i x_i) = f_i. */
mg_status mg_fold(mg_hierarchy *H, const double *rho_dev, const double *dirichlet_dev, double *f_dev);

/* `passes` red-black Gauss-Seidel passes (red = (i+j+k) even first) on
 * level l for the system L x = f (Sec. 2); x in/out. */
mg_status mg_smooth(mg_hierarchy *H, int32_t level, int32_t order, double *x_dev, const double *f_dev,
                    int32_t passes);

/* r = L x - f on level l (Sec. 2 step 2). */
mg_status mg_residual(mg_hierarchy *H, int32_t level, int32_t order, const double *x_dev, const double *f_dev,
                      double *r_dev);

/* Coarse right-hand side f_c = -R1(L x - f) on level l+1 (Sec. 2 steps 2-5):
 * the sum over active children divided by 8, on active coarse cells. */
mg_status mg_restrict_residual(mg_hierarchy *H, int32_t level, int32_t order, const double *x_dev,
                               const double *f_dev, double *fc_dev);

/* x += P2(xc) on active cells of level l, xc on level l+1 (Sec. 2 steps
 * 6-7; coarse values off the coarse domain count as 0).  x in/out. */
mg_status mg_prolong(mg_hierarchy *H, int32_t level, int32_t order, const double *xc_dev, double *x_dev);

/* One multigrid iteration MG(0) (Sec. 2) on the folded finest system,
 * x in/out (finest level), f from mg_fold. */
mg_status mg_vcycle(mg_hierarchy *H, int32_t order, double *x_dev, const double *f_dev);

/*
 * Run the finest-level smoother kernel `launches` times on the hierarchy's
 * own buffers (contents left by the last solve), back to back on the
 * hierarchy stream, for bandwidth measurement (with fuse_passes, each launch
 * is the fused kernel doing two passes).  Host returns at once.
 */
mg_status mg_time_smoother(mg_hierarchy *H, int32_t order, int32_t launches);

/*
 * Duration of one kind of finest-level red-black launch inside later solves
 * (FP64, or FP32 in a mixed solve).  enable selects the kind, clears the
 * record and launches each such pass with a pair of HIP events that take the
 * kernel's own start and end times (hipExtLaunchKernel), up to 1024
 * launches: 1 = the plain passes (those that neither form the input norm,
 * nor the residual, nor apply the prolongation), 2 = the last pre-smoothing
 * pass that also forms the residual and its restriction (fuse_restrict), 3 =
 * the first post-smoothing pass that applies the prolongation, 4 = the first
 * pre-smoothing pass that also forms the residual norm of its input (FP64).
 * A launch of a cycle that the device stop test halted is dropped from the
 * record; enable = 0 stops recording.  Both synchronise the stream first.
 * MG_ERR_ARG for another enable value or with use_graph set (a captured
 * cycle records no events).
 */
mg_status mg_kernel_timing(mg_hierarchy *H, int32_t enable);

/* Synchronise the stream; *ms_total = the summed durations of the recorded
 * launches, *launches = their count. */
mg_status mg_kernel_timing_read(mg_hierarchy *H, double *ms_total, int32_t *launches);

/* The stream the hierarchy enqueues on (as void*). */
void *mg_stream(const mg_hierarchy *H);

/* ---------------- batched solver ---------------- */
/* Many independent masked grids (AMR-level patches of uneven size and depth)
 * solved together: each patch has its own hierarchy, operators, order switch
 * (Sec. 4) and stop test exactly as in mg_solve (Sec. 2-4), and gets bit for
 * bit the result mg_solve gives it.  One multigrid cycle of all unconverged
 * patches runs as one program of launches on the batch stream, each launch
 * one phase of the cycle (a red-black pass on level l, a restriction, the
 * small levels) over the work items of every patch that reaches it.  A
 * cycle's first finest pass runs ahead of the host's decisions and also
 * forms the residual norm of its input (the norm-forming pass of mg_solve),
 * so the host reads all patch norms once per cycle, between that pass and
 * the rest of the cycle, and a patch that stops keeps that input.  Options the programs
 * do not cover (odd finest-level pass counts per cycle, n_post == 0, a
 * zero-pass relaxation from zero) run each patch's own captured cycle in
 * lockstep instead.  use_graph = 1 replays each program from a captured
 * graph.  Calls on one batch must not overlap. */
typedef struct mg_batch mg_batch; /* opaque */

/*
 * Build the hierarchies of n patches.
 *   masks_dev : n device pointers to int8 masks (+1/-1, inactive outer layer).
 *   dims      : 3n host ints (nx, ny, nz per patch).   h: n host cell widths.
 *   opt       : NULL = defaults; precision must be MG_FP64.
 * Errors as mg_create_hierarchy (the first failing patch).
 */
mg_status mg_create_batch(int32_t n, const int8_t *const *masks_dev, const int32_t *dims, const double *h,
                          const mg_options *opt, void *stream, mg_batch **out);

/*
 * Solve every patch to ||r||_2 <= tol ||r(phi=0)||_2 (per patch), each with its
 * own runtime order switch (Sec. 4) and first-order hold.
 *   rho_dev, phi_dev : n device pointers each (phi: guess in, solution out on
 *                      active cells).  dirichlet_dev: NULL, or n device
 *                      pointers (entries may be NULL).
 *   infos : NULL or n records.   ms_out: NULL or the wall time on the stream.
 * Returns MG_OK if every patch converged, else the worst status (negative
 * errors before MG_NOT_CONVERGED).
 */
mg_status mg_solve_batch(mg_batch *B, const double *const *rho_dev, double *const *phi_dev,
                         const double *const *dirichlet_dev, double tol, mg_solve_info *infos, double *ms_out);

/* Release the batch and every patch hierarchy (NULL is a no-op). */
void mg_destroy_batch(mg_batch *B);

/* Number of patches; work items of the largest launch of the cycle programs,
 * and launches per cycle in boundary order `order` (1 or 2; the pass that
 * forms the norm, the norm's sum and the rest of the cycle), both 0 when the
 * batch runs on the per-patch lockstep engine only. */
int32_t mg_batch_size(const mg_batch *B);
int32_t mg_batch_grid(const mg_batch *B);
int32_t mg_batch_phases(const mg_batch *B, int32_t order);

/* Re-run the host-side validation of the phase programs' tables (run once at
 * creation, before any phase kernel): every work item's patch, level, item
 * index and selector against the hierarchy it refers to, launch ranges,
 * partial-sum offsets and small-level LDS sizes.  Returns the number of
 * violations (0 for a valid batch; -1 for NULL) and copies a description
 * of the first ones into msg (capacity len, may be NULL). */
int32_t mg_batch_validate(const mg_batch *B, char *msg, int32_t len);

/* Select the engine of later solves: 1 the phase programs, one launch per
 * phase (the default where they exist; MG_ERR_ARG if they do not); 2 the
 * same programs as phases of one persistent cooperative launch per V-cycle
 * (the cycle in each boundary order in use, then the next cycle's first
 * finest pass with the norm of its input; grid-wide barriers between
 * phases; MG_ERR_ARG where the device cannot run it); 0 the per-patch
 * lockstep cycles.  All give the same results bit for bit. */
mg_status mg_batch_set_engine(mg_batch *B, int32_t phased);

/* ---------------- one-way nested levels (AMR) ----------------
 * A refined level is solved after the next coarser one (Sec. 3, one-way
 * interface; Sec. 5.1): its Dirichlet values are the coarser potential
 * interpolated linearly to its boundary faces, and the gradient of the
 * potential takes the values it needs beyond the level from the coarser level
 * the same way (Fig. "force-ramses").  A level is a box array (nz, ny, nx) of
 * cells of width h whose lower corner is at origin = (x0, y0, z0) (host, 3
 * doubles); cell (i, j, k) is centred at origin + ((i, j, k) + 1/2) h.
 * Linear interpolation between cell centres is trilinear.  Both calls only
 * enqueue on `stream` (void* hipStream_t, NULL = default).
 */

/*
 * Dirichlet field of a refined patch whose outer layer is its boundary and
 * whose interior is active, in the solver's cell-centred form (the face value
 * between active i and inactive j is (B_i + B_j) / 2): interior cells get the
 * interpolated coarser potential at their centre, a frame cell sharing a face
 * with one interior cell gets 2 g - B_i (g = the interpolated potential at
 * that face's centre), edge and corner frame cells 0.
 *   phi_c_dev: coarser level (cnz, cny, cnx), cell width hc, corner origin_c.
 *   b_dev:     output (nz, ny, nx), cell width hf, corner origin_f.
 * MG_ERR_ARG for null pointers, dims below 3, h <= 0, or when the coarser
 * array does not hold the interpolation stencil of every point used.
 */
mg_status mg_amr_dirichlet(const double *phi_c_dev, int32_t cnx, int32_t cny, int32_t cnz, double hc,
                           const double *origin_c, int32_t nx, int32_t ny, int32_t nz, double hf,
                           const double *origin_f, double *b_dev, void *stream);

/*
 * Gradient of phi on the active cells (mask == +1) of a level by the 5-point
 * difference (Sec. 5.1): d/dx phi = (4/3)(phi[i+1] - phi[i-1])/(2h)
 * - (1/3)(phi[i+2] - phi[i-2])/(4h), likewise in y and z.  A value at a cell
 * that is not an active cell of the level comes from the coarser level
 * (phi_c_dev, may be NULL) at that cell's centre; with no coarser level, from
 * bnd_dev (the level's Dirichlet field, may be NULL) inside the array, NaN
 * beyond.  grad_dev: 3 * nz * ny * nx doubles, components x, y, z one after
 * the other; inactive cells get 0.  MG_ERR_ARG as above, or when the coarser
 * array does not cover the level plus a 2-cell margin.
 */
mg_status mg_amr_grad5(const double *phi_dev, const int8_t *mask_dev, int32_t nx, int32_t ny, int32_t nz, double h,
                       const double *origin, const double *phi_c_dev, int32_t cnx, int32_t cny, int32_t cnz,
                       double hc, const double *origin_c, const double *bnd_dev, double *grad_dev, void *stream);

/* ---------------- learned first guess (U-Net) ----------------
 * The iteration of Sec. 2 converges from any first guess, and the paper's
 * convergence is insensitive to it (Sec. 2, Sec. 6); these calls produce a
 * guess phi0 from (rho, mask, B) with a 3D U-Net, then mg_solve takes phi0 as
 * its initial phi.  The stopping target (tol times the zero-guess residual
 * norm) is the same for every guess.
 *
 * Network: 4 resolutions with 16, 32, 64, 128 channels; per stage two 3x3x3
 * convolutions (zero padding) each followed by ReLU; 2x2x2 mean pooling;
 * nearest up-sampling concatenated (up-sampled channels first) with the
 * encoder tensor of the same resolution; a 1x1x1 head to one channel.
 * Convolutions run on the BF16 matrix cores with FP32 accumulation; tensors
 * are BF16 channels-last; master weights, gradients and AdamW moments are
 * FP32.
 * Input (16 channels): rho / s on active cells (0 elsewhere), the mask
 * (+1/-1), B / s, zeros; s = root mean square of rho over the sample's active
 * cells (1 if zero).  Output: phi0 = s * y / 256 on active cells, 0 elsewhere.
 * Parameters (float32, mg_unet_num_params of them): per layer in the order
 * enc1a enc1b enc2a enc2b enc3a enc3b mid4a mid4b dec3a dec3b dec2a dec2b
 * dec1a dec1b, weights [27][cout][cin] (tap = 9(dz+1) + 3(dy+1) + (dx+1))
 * then bias [cout]; last the head weights [16] and bias [1].
 * A network object is not re-entrant; all its work goes to its stream.
 */
typedef struct mg_unet mg_unet; /* opaque */

/* Create a network with He-normal weights drawn from `seed` (zero biases).
 * alloc: NULL = hipMalloc.  stream: 0 = a stream of its own. */
mg_status mg_unet_create(uint64_t seed, const mg_allocator *alloc, void *stream, mg_unet **out);
void mg_unet_destroy(mg_unet *U);
int64_t mg_unet_num_params(const mg_unet *U);
void *mg_unet_stream(const mg_unet *U);
/* AdamW steps taken since the parameters were last set. */
int32_t mg_unet_step(const mg_unet *U);

/* Copy parameters in / out (host float32, count = mg_unet_num_params).
 * Setting resets the AdamW moments and step.  Synchronous. */
mg_status mg_unet_set_params(mg_unet *U, const float *params_host, int64_t count);
mg_status mg_unet_get_params(mg_unet *U, float *params_host, int64_t count);
/* Gradient of the loss of the last mg_unet_loss_grad / mg_unet_train_step. */
mg_status mg_unet_get_grads(mg_unet *U, float *grads_host, int64_t count);

/* Save / load parameters and AdamW state as a safetensors file (float32
 * tensors "params", "adam_m", "adam_v"; metadata "step").  Loading a file
 * with "params" only resets the optimizer.  MG_ERR_ARG on I/O or shape
 * mismatch. */
mg_status mg_unet_save(mg_unet *U, const char *path);
mg_status mg_unet_load(mg_unet *U, const char *path);

/*
 * Loss and gradient for a batch of n samples: loss = mean over all active
 * cells of the batch of (y - 256 phi_target / s_n)^2.
 *   rho_dev, dirichlet_dev (NULL = 0), phi_target_dev : float64 (n, nz, ny, nx);
 *   mask_dev : int8 (n, nz, ny, nx).  nx, ny, nz multiples of 8.
 *   loss_out : host, receives the loss (the call synchronises the stream).
 */
mg_status mg_unet_loss_grad(mg_unet *U, int32_t n, const double *rho_dev, const int8_t *mask_dev,
                            const double *dirichlet_dev, const double *phi_target_dev, int32_t nx, int32_t ny,
                            int32_t nz, double *loss_out);

/* mg_unet_loss_grad followed by one AdamW update (beta1 0.9, beta2 0.999,
 * eps 1e-8, decoupled weight decay, bias-corrected moments).  loss_out may be
 * NULL (no synchronisation). */
mg_status mg_unet_train_step(mg_unet *U, int32_t n, const double *rho_dev, const int8_t *mask_dev,
                             const double *dirichlet_dev, const double *phi_target_dev, int32_t nx, int32_t ny,
                             int32_t nz, float lr, float weight_decay, double *loss_out);

/*
 * Copy one tensor the network keeps between layers (BF16, channels-last, for
 * the batch shape of the last mg_unet_loss_grad / mg_unet_train_step /
 * mg_unet_infer call) into dst_dev, for per-layer checks of the chain rule
 * that mg_unet_loss_grad applies layer by layer.  kind:
 *   MG_UNET_ACT       index 0..13: layer output after ReLU (layer order above)
 *   MG_UNET_ACT_GRAD  index 0..13: after a loss_grad, the loss gradient of the
 *                     layer's output with the ReLU applied (zero where the
 *                     output is not positive), i.e. of its pre-activation
 *   MG_UNET_POOL      index 0..2: the pooled encoder outputs (levels 2..4)
 *   MG_UNET_POOL_GRAD index 0..2: after a loss_grad, their loss gradients
 *   MG_UNET_INPUT     index 0: the packed 16-channel input
 *   MG_UNET_CAT_GRAD  index 0: after a loss_grad, the gradient of the last
 *                     concatenated input differentiated (that of dec3a)
 * count must equal the tensor's element count (MG_ERR_ARG otherwise, also
 * when the tensor does not exist, e.g. a gradient after an inference).  The
 * copy is enqueued on the network's stream and the call synchronises it.
 */
enum { MG_UNET_ACT = 0, MG_UNET_ACT_GRAD = 1, MG_UNET_POOL = 2, MG_UNET_POOL_GRAD = 3, MG_UNET_INPUT = 4,
       MG_UNET_CAT_GRAD = 5 };
mg_status mg_unet_tensor(mg_unet *U, int32_t kind, int32_t index, void *dst_dev, int64_t count);

/*
 * First guess for one problem (nz, ny, nx), written to phi0_dev (float64,
 * every cell; 0 off the active set).  The network runs on the 1/stride grid
 * (stride 1, 2, 4 or 8; dims multiples of 8 * stride): each coarse cell takes
 * the mean of rho over its active fine cells, +1 when more than half of them
 * are active, and the mean of B; the output is brought back to the fine grid
 * by repeated linear up-sampling by 2 (per axis 3/4 of the parent, 1/4 of the
 * next coarse cell, the edge cell repeated past the array end).  Enqueued on
 * the network's stream; no synchronisation.
 */
mg_status mg_unet_infer(mg_unet *U, const double *rho_dev, const int8_t *mask_dev, const double *dirichlet_dev,
                        int32_t nx, int32_t ny, int32_t nz, int32_t stride, double *phi0_dev);

/*
 * Coarse copy of a problem, for an interpolated first guess: the problem
 * solved on the stride-times coarser grid (Sec. 6 compares against
 * interpolated starts).  mask_c: +1 when more than half of the block is
 * active, the outermost coarse layer -1; rho_c: mean of rho over the active
 * cells of the block (0 if none); dirichlet_c: mean of B (written only if
 * dirichlet_dev is not NULL).  Dims must be multiples of stride (>= 2).
 */
mg_status mg_coarsen_problem(const double *rho_dev, const int8_t *mask_dev, const double *dirichlet_dev, int32_t nx,
                             int32_t ny, int32_t nz, int32_t stride, double *rho_c_dev, int8_t *mask_c_dev,
                             double *dirichlet_c_dev, void *stream);

/* phi = linear up-sampling by 2 of phi_c (dims nxc, nyc, nzc) on the active
 * cells of mask (dims 2nxc, 2nyc, 2nzc), 0 elsewhere. */
mg_status mg_upsample_guess(const double *phi_c_dev, int32_t nxc, int32_t nyc, int32_t nzc, const int8_t *mask_dev,
                            double *phi_dev, void *stream);

/* ---- network kernels, exported for tests (BF16 channels-last tensors) ---- */
/* out = [ReLU](conv3x3x3(concat(up2?(in_a), in_b)) + bias).  in_a: ca
 * channels, read at half resolution (nearest) when up_a; in_b: cb channels
 * or NULL; w: BF16 [27][cout][ca+cb]; bias: float32 [cout] or NULL.  ca, cb
 * multiples of 8, cout of 16. */
mg_status mg_nn_conv3d_fwd(const void *in_a, int32_t ca, int32_t up_a, const void *in_b, int32_t cb, const void *w,
                           const float *bias, void *out, int32_t cout, int32_t relu, int32_t n, int32_t d, int32_t h,
                           int32_t wd, void *stream);
/* dw[27][cout][ca+cb] += sum_v dout[v][co] x[v + tap][ci]; dbias[cout] (or
 * NULL) += sum_v dout[v][co] (float32, accumulated).  ca+cb in {16, 32, 48,
 * 64, 96, 128, 192}. */
mg_status mg_nn_conv3d_bwd_weight(const void *dout, int32_t cout, const void *in_a, int32_t ca, int32_t up_a,
                                  const void *in_b, int32_t cb, float *dw, float *dbias, int32_t n, int32_t d,
                                  int32_t h, int32_t wd, void *stream);
/* wt[26 - tap][ci][co] = w[tap][co][ci] (the input-gradient convolution's weights). */
mg_status mg_nn_weight_flip(const void *w, int32_t cout, int32_t cin, void *wt, void *stream);
/* dy[i] = 0 where y[i] <= 0. */
mg_status mg_nn_relu_bwd(void *dy, const void *y, int64_t count, void *stream);
/* 2x2x2 mean pooling of (n, d, h, wd, c); and its gradient, din += dout / 8. */
mg_status mg_nn_pool2(const void *in, void *out, int32_t c, int32_t n, int32_t d, int32_t h, int32_t wd, void *stream);
mg_status mg_nn_pool2_bwd(const void *dout, void *din, int32_t c, int32_t n, int32_t d, int32_t h, int32_t wd,
                          void *stream);
/* Gradient of a concatenated input (n, d, h, wd, ca+cb): dup (half
 * resolution, ca channels) = sum over the 8 children, dskip = the last cb
 * channels. */
mg_status mg_nn_split_grad(const void *dx, int32_t ca, int32_t cb, void *dup, void *dskip, int32_t n, int32_t d,
                           int32_t h, int32_t wd, void *stream);
/* AdamW on float32 params (optional BF16 copy refreshed). */
mg_status mg_nn_adamw(float *param, void *param_bf16, const float *grad, float *m, float *v, int64_t count, float lr,
                      float beta1, float beta2, float eps, float weight_decay, int32_t step, void *stream);
/* Writes the 16 x 16 product of the matrix-core self-test (row-major float32)
 * to out_dev: a[m][k] = (3m + k) mod 7 - 3, b[k][n] = (5k + 2n) mod 9 - 4,
 * k < 32. */
mg_status mg_nn_mfma_selftest(float *out_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MG_H */
