/*
 * Plain FP64 CPU oracle for the masked multigrid Poisson solver of
 * Guillet & Teyssier, "A Simple Multigrid Scheme for Solving the Poisson
 * Equation with Arbitrary Domain Boundaries" (arXiv:1104.1703).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  The GPU library does
 * not include, link or call it; it shares no header or helper with it.
 *
 * Every routine follows one passage of the paper, cited in its comment:
 *   - Sec. 2, enumerated multigrid iteration (smooth, residual, restrict,
 *     coarse problem with zero boundary values, prolong, correct, smooth);
 *   - Sec. 2, 7-point Laplacian and red-black Gauss-Seidel;
 *   - Sec. 2, Fig. "operators": R1 restriction (average of the children)
 *     and P2 prolongation (trilinear interpolation);
 *   - Sec. 3: mask colouring +1/-1, recursive R1 averaging of the mask,
 *     domain {m > 0}, ghost value linearly extrapolated from the cell and the
 *     boundary value at the zero crossing of the linearly interpolated mask,
 *     direction by direction (Figs. "stencil" and "ghost");
 *   - Sec. 4: first-order ("NGP") coarse boundary, cells with m < 1 pinned to
 *     zero; runtime switch when ||r_{n+1}|| / ||r_n|| > eta, held for the
 *     next 10 solves.
 *
 * Readings where the paper is silent (stated once here, used throughout):
 *   - Masks are kept as exact integer counts c of active finest-level
 *     descendants: m = 2c/8^l - 1, so "m > 0" is 2c > 8^l and "m = 1" is
 *     c = 8^l.  Out-of-array cells have m = -1.
 *   - At the finest level the boundary lies on the face between an active
 *     and an inactive cell (theta = 1/2); the Dirichlet value on that face is
 *     the average of a caller-supplied cell-centred field B on both sides.
 *   - Coarse levels carry boundary value 0 (the coarse correction problem).
 *     Second order: theta_ij = m_i / (m_i - m_j).  First order: theta = 1
 *     (the pinned neighbour's centre is the boundary).
 *   - Red cells ((i+j+k) even, level-local indices) are relaxed first.
 *   - The coarse initial guess is zero; the deepest non-empty level is
 *     relaxed n_coarse times.
 *   - Residual restriction sums only active children, divides by 8 and
 *     changes sign (the coarse right-hand side of Delta dPhi = -r).
 *   - Prolongation uses zero for coarse values outside the coarse domain.
 *   - Stop test ||r||_2 <= tol * ||r(phi = 0)||_2 over active finest cells.
 *   - Reductions: sum over each z-plane in (j, i) order, then over planes in
 *     k order; so the OpenMP build equals the serial one bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXL 16

typedef struct {
    int n_pre, n_post, n_cycles, n_coarse, max_cycles;
    int bc_order;       /* 0 = automatic switch, 1 = first order, 2 = second order */
    double eta;         /* convergence-rate threshold of the switch */
    int hold;           /* solves kept in first order after a switch */
} orc_opts;

typedef struct {
    int cycles, order_used, switched_at, status;
    double r_ref, r0, r_final;
    double history[257];
} orc_info;

typedef struct {
    int nlev_geom;                 /* levels that exist geometrically */
    int nlev[3];                   /* levels used per order (index 1, 2) */
    int nx[ORC_MAXL], ny[ORC_MAXL], nz[ORC_MAXL];
    double h[ORC_MAXL];
    int64_t *cnt[ORC_MAXL];        /* active finest descendants */
    uint8_t *act[3][ORC_MAXL];     /* active flags per order */
    double *x[ORC_MAXL], *f[ORC_MAXL], *r[ORC_MAXL]; /* work arrays, levels >= 1 */
    double *r0;                    /* finest-level residual scratch */
    int hold_left;                 /* remaining solves forced to first order */
} orc_h;

static size_t ncell(const orc_h *H, int l) { return (size_t)H->nx[l] * H->ny[l] * H->nz[l]; }
static size_t idx(const orc_h *H, int l, int i, int j, int k) {
    return ((size_t)k * H->ny[l] + j) * H->nx[l] + i;
}
static int inside(const orc_h *H, int l, int i, int j, int k) {
    return i >= 0 && j >= 0 && k >= 0 && i < H->nx[l] && j < H->ny[l] && k < H->nz[l];
}
static int64_t nfine(int l) { return (int64_t)1 << (3 * l); }  /* 8^l */

/* Active test (Sec. 3 domain {m > 0}; Sec. 4 first order {m = 1}). */
static int active(const orc_h *H, int l, int order, int i, int j, int k) {
    if (!inside(H, l, i, j, k)) return 0;
    return H->act[order][l][idx(H, l, i, j, k)];
}

static const int NB[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

/*
 * theta for the face between active cell i and inactive neighbour j
 * (Sec. 3, Fig. "ghost": zero crossing of the linearly interpolated mask).
 */
static double theta(const orc_h *H, int l, int order, int i, int j, int k, int in, int jn, int kn) {
    if (l == 0) return 0.5;
    if (order == 1) return 1.0;
    int64_t N = nfine(l);
    int64_t ci = H->cnt[l][idx(H, l, i, j, k)];
    int64_t cj = inside(H, l, in, jn, kn) ? H->cnt[l][idx(H, l, in, jn, kn)] : 0;
    double mi = (double)(2 * ci - N) / (double)N;
    double mj = (double)(2 * cj - N) / (double)N;
    return mi / (mi - mj);
}

/*
 * Ghost-modified 7-point operator applied at active cell (i,j,k)
 * (Sec. 2 Laplacian; Sec. 3 ghost value).  Each neighbour contributes
 * (phi_j - phi_i); an inactive neighbour is replaced by the ghost
 * (g - (1 - theta) phi_i) / theta, g the boundary value on that face.
 * Returns the Laplacian times h^2.  If xi_override is used the centre value
 * is taken from it (Gauss-Seidel needs the operator as a function of x_i).
 */
static double lap_h2(const orc_h *H, int l, int order, const double *x, const double *B,
                     int i, int j, int k, double xi) {
    double s = 0.0;
    for (int q = 0; q < 6; q++) {
        int in = i + NB[q][0], jn = j + NB[q][1], kn = k + NB[q][2];
        if (active(H, l, order, in, jn, kn)) {
            s += x[idx(H, l, in, jn, kn)] - xi;
        } else {
            double th = theta(H, l, order, i, j, k, in, jn, kn);
            double g = 0.0;
            if (l == 0 && B) g = 0.5 * (B[idx(H, l, i, j, k)] + B[idx(H, l, in, jn, kn)]);
            double ghost = (g - (1.0 - th) * xi) / th;
            s += ghost - xi;
        }
    }
    return s;
}

/*
 * Diagonal of the operator (times -h^2): the operator is affine in x_i with
 * slope -d_i/h^2 where d_i = #active neighbours + sum over inactive ones of
 * 1/theta.  Gauss-Seidel solves the cell's own equation for x_i.
 */
static double diag(const orc_h *H, int l, int order, int i, int j, int k) {
    double d = 0.0;
    for (int q = 0; q < 6; q++) {
        int in = i + NB[q][0], jn = j + NB[q][1], kn = k + NB[q][2];
        if (active(H, l, order, in, jn, kn)) d += 1.0;
        else d += 1.0 / theta(H, l, order, i, j, k, in, jn, kn);
    }
    return d;
}

/* ---------------- hierarchy (Sec. 2 Fig. "hierarchy"; Sec. 3 mask) ---------------- */

void orc_destroy(orc_h *H) {
    if (!H) return;
    for (int l = 0; l < ORC_MAXL; l++) {
        free(H->cnt[l]);
        for (int o = 0; o < 3; o++) free(H->act[o][l]);
        free(H->x[l]); free(H->f[l]); free(H->r[l]);
    }
    free(H->r0);
    free(H);
}

/*
 * Build the hierarchy from the finest mask (values +1 / -1).
 * Coarsen while every dimension is even and the next level keeps every
 * dimension >= min_dim.  Returns NULL on invalid input, including a mask
 * without an active cell.
 */
orc_h *orc_create(const int8_t *mask, int nx, int ny, int nz, double h, int min_dim) {
    if (!mask || nx < 1 || ny < 1 || nz < 1 || !(h > 0)) return NULL;
    orc_h *H = (orc_h *)calloc(1, sizeof(orc_h));
    H->nx[0] = nx; H->ny[0] = ny; H->nz[0] = nz; H->h[0] = h;
    int L = 1;
    while (L < ORC_MAXL) {
        int a = H->nx[L - 1], b = H->ny[L - 1], c = H->nz[L - 1];
        if (a % 2 || b % 2 || c % 2) break;
        if (a / 2 < min_dim || b / 2 < min_dim || c / 2 < min_dim) break;
        H->nx[L] = a / 2; H->ny[L] = b / 2; H->nz[L] = c / 2; H->h[L] = 2.0 * H->h[L - 1];
        L++;
    }
    H->nlev_geom = L;
    /* finest counts: 1 where m = +1 */
    H->cnt[0] = (int64_t *)calloc(ncell(H, 0), sizeof(int64_t));
    for (size_t p = 0; p < ncell(H, 0); p++) H->cnt[0][p] = (mask[p] == 1) ? 1 : 0;
    /* coarse counts: R1 averaging of the mask, kept as integer sums */
    for (int l = 1; l < L; l++) {
        H->cnt[l] = (int64_t *)calloc(ncell(H, l), sizeof(int64_t));
        for (int k = 0; k < H->nz[l]; k++)
            for (int j = 0; j < H->ny[l]; j++)
                for (int i = 0; i < H->nx[l]; i++) {
                    int64_t s = 0;
                    for (int c = 0; c < 8; c++)
                        s += H->cnt[l - 1][idx(H, l - 1, 2 * i + (c & 1), 2 * j + ((c >> 1) & 1), 2 * k + (c >> 2))];
                    H->cnt[l][idx(H, l, i, j, k)] = s;
                }
    }
    /* an empty domain has no unknowns: rejected, as the GPU library does */
    {
        size_t na0 = 0;
        for (size_t p = 0; p < ncell(H, 0); p++) na0 += (size_t)H->cnt[0][p];
        if (na0 == 0) {
            orc_destroy(H);
            return NULL;
        }
    }
    /* active sets per order */
    for (int o = 1; o <= 2; o++) {
        H->nlev[o] = 0;
        for (int l = 0; l < L; l++) {
            H->act[o][l] = (uint8_t *)calloc(ncell(H, l), 1);
            int64_t N = nfine(l);
            size_t na = 0;
            for (size_t p = 0; p < ncell(H, l); p++) {
                int64_t c = H->cnt[l][p];
                int a;
                if (l == 0) a = (c == 1);
                else if (o == 2) a = (2 * c > N);   /* m > 0 */
                else a = (c == N);                  /* m = 1 */
                H->act[o][l][p] = (uint8_t)a;
                na += a;
            }
            if (na > 0 && H->nlev[o] == l) H->nlev[o] = l + 1;
        }
    }
    for (int l = 1; l < L; l++) {
        H->x[l] = (double *)calloc(ncell(H, l), sizeof(double));
        H->f[l] = (double *)calloc(ncell(H, l), sizeof(double));
        H->r[l] = (double *)calloc(ncell(H, l), sizeof(double));
    }
    H->r0 = (double *)calloc(ncell(H, 0), sizeof(double));
    return H;
}

int orc_nlevels(const orc_h *H, int order) { return (order == 1 || order == 2) ? H->nlev[order] : H->nlev_geom; }

void orc_level_dims(const orc_h *H, int l, int *dims) { dims[0] = H->nx[l]; dims[1] = H->ny[l]; dims[2] = H->nz[l]; }

void orc_level_counts(const orc_h *H, int l, int64_t *out) { memcpy(out, H->cnt[l], ncell(H, l) * sizeof(int64_t)); }

void orc_level_active(const orc_h *H, int l, int order, uint8_t *out) {
    memcpy(out, H->act[order][l], ncell(H, l));
}

void orc_level_diag(const orc_h *H, int l, int order, double *out) {
    for (int k = 0; k < H->nz[l]; k++)
        for (int j = 0; j < H->ny[l]; j++)
            for (int i = 0; i < H->nx[l]; i++) {
                size_t p = idx(H, l, i, j, k);
                out[p] = H->act[order][l][p] ? diag(H, l, order, i, j, k) : 0.0;
            }
}

int orc_get_hold(const orc_h *H) { return H->hold_left; }
void orc_set_hold(orc_h *H, int v) { H->hold_left = v; }

/* ---------------- operators ---------------- */

/*
 * Red-black Gauss-Seidel (Sec. 2): `passes` full passes, each relaxing the
 * colour (i+j+k) even, then odd.  Relaxing cell i sets x_i so that the
 * cell's own equation  L x = rhs  holds with the neighbours fixed.  Cells of
 * one colour only read the other colour, so the planes of one colour are
 * independent (parallel loop).  B is used on the finest level only.
 */
void orc_smooth(const orc_h *H, int l, int order, double *x, const double *rhs, const double *B, int passes) {
    double h2 = H->h[l] * H->h[l];
    for (int p = 0; p < passes; p++)
        for (int colour = 0; colour < 2; colour++) {
#pragma omp parallel for schedule(static)
            for (int k = 0; k < H->nz[l]; k++)
                for (int j = 0; j < H->ny[l]; j++)
                    for (int i = 0; i < H->nx[l]; i++) {
                        if (((i + j + k) & 1) != colour) continue;
                        if (!active(H, l, order, i, j, k)) continue;
                        size_t c = idx(H, l, i, j, k);
                        /* L(x_i) = (a - d x_i)/h^2 with a = lap_h2 at x_i = 0 */
                        double a = lap_h2(H, l, order, x, B, i, j, k, 0.0);
                        double d = diag(H, l, order, i, j, k);
                        x[c] = (a - h2 * rhs[c]) / d;
                    }
        }
}

/* Residual r = L x - rhs on active cells, 0 elsewhere (Sec. 2 step 2). */
void orc_residual(const orc_h *H, int l, int order, const double *x, const double *rhs, const double *B, double *r) {
    double ih2 = 1.0 / (H->h[l] * H->h[l]);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < H->nz[l]; k++)
        for (int j = 0; j < H->ny[l]; j++)
            for (int i = 0; i < H->nx[l]; i++) {
                size_t c = idx(H, l, i, j, k);
                if (!active(H, l, order, i, j, k)) { r[c] = 0.0; continue; }
                r[c] = lap_h2(H, l, order, x, B, i, j, k, x[c]) * ih2 - rhs[c];
            }
}

/*
 * R1 restriction of the residual to level l+1 (Sec. 2 Fig. "operators"),
 * giving the coarse right-hand side of  Delta_c dPhi = -r_c  (step 5).
 * Only active children contribute; inactive coarse cells get 0.
 */
void orc_restrict(const orc_h *H, int l, int order, const double *r, double *fc) {
    int L = l + 1;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < H->nz[L]; k++)
        for (int j = 0; j < H->ny[L]; j++)
            for (int i = 0; i < H->nx[L]; i++) {
                size_t C = idx(H, L, i, j, k);
                if (!active(H, L, order, i, j, k)) { fc[C] = 0.0; continue; }
                double s = 0.0;
                for (int c = 0; c < 8; c++) {
                    int a = 2 * i + (c & 1), b = 2 * j + ((c >> 1) & 1), e = 2 * k + (c >> 2);
                    if (active(H, l, order, a, b, e)) s += r[idx(H, l, a, b, e)];
                }
                fc[C] = -s / 8.0;
            }
}

/*
 * P2 prolongation and correction (Sec. 2 steps 6-7, Fig. "operators"):
 * each active fine cell adds the trilinear interpolant of the coarse
 * correction at its centre.  Along an axis the fine centre sits 1/4 coarse
 * cell from its parent's centre towards the side given by its child offset,
 * so the weights are 3/4 (parent) and 1/4 (next coarse cell on that side).
 * Coarse values outside the coarse domain count as 0 (dPhi_c = 0 there).
 */
void orc_prolong(const orc_h *H, int l, int order, const double *xc, double *x) {
    int L = l + 1;
    static const double w[2] = {0.75, 0.25};
#pragma omp parallel for schedule(static)
    for (int k = 0; k < H->nz[l]; k++)
        for (int j = 0; j < H->ny[l]; j++)
            for (int i = 0; i < H->nx[l]; i++) {
                if (!active(H, l, order, i, j, k)) continue;
                int I = i / 2, J = j / 2, K = k / 2;
                int sx = (i & 1) ? 1 : -1, sy = (j & 1) ? 1 : -1, sz = (k & 1) ? 1 : -1;
                double s = 0.0;
                for (int c = 0; c < 2; c++)
                    for (int b = 0; b < 2; b++)
                        for (int a = 0; a < 2; a++) {
                            int ci = I + a * sx, cj = J + b * sy, ck = K + c * sz;
                            double v = active(H, L, order, ci, cj, ck) ? xc[idx(H, L, ci, cj, ck)] : 0.0;
                            s += w[a] * w[b] * w[c] * v;
                        }
                x[idx(H, l, i, j, k)] += s;
            }
}

/* Sum of squares over a level with the fixed plane-then-total order. */
static double norm2(const orc_h *H, int l, const double *r) {
    int nz = H->nz[l];
    double *plane = (double *)calloc((size_t)nz, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++) {
        double s = 0.0;
        for (int j = 0; j < H->ny[l]; j++)
            for (int i = 0; i < H->nx[l]; i++) {
                double v = r[idx(H, l, i, j, k)];
                s += v * v;
            }
        plane[k] = s;
    }
    double t = 0.0;
    for (int k = 0; k < nz; k++) t += plane[k];
    free(plane);
    return sqrt(t);
}

/*
 * One multigrid iteration at level l (Sec. 2, enumerated recipe):
 * pre-smooth, residual, restrict, coarse correction by n_cycles iterations
 * started from zero (zero boundary values on the coarse domain), prolong and
 * correct, post-smooth.  The deepest level is relaxed n_coarse times.
 */
static void mg_level(orc_h *H, int l, int order, double *x, const double *rhs, const double *B, const orc_opts *o) {
    int last = H->nlev[order] - 1;
    if (l == last) {
        orc_smooth(H, l, order, x, rhs, B, o->n_coarse);
        return;
    }
    orc_smooth(H, l, order, x, rhs, B, o->n_pre);
    double *r = (l == 0) ? H->r0 : H->r[l];
    orc_residual(H, l, order, x, rhs, B, r);
    orc_restrict(H, l, order, r, H->f[l + 1]);
    memset(H->x[l + 1], 0, ncell(H, l + 1) * sizeof(double));
    for (int c = 0; c < o->n_cycles; c++) mg_level(H, l + 1, order, H->x[l + 1], H->f[l + 1], NULL, o);
    orc_prolong(H, l, order, H->x[l + 1], x);
    orc_smooth(H, l, order, x, rhs, B, o->n_post);
}

/* One iteration on the finest level, exposed for per-cycle comparisons. */
void orc_vcycle(orc_h *H, int order, double *phi, const double *rho, const double *B, const orc_opts *o) {
    mg_level(H, 0, order, phi, rho, B, o);
}

/* ||L phi - rho||_2 over the active finest cells. */
double orc_residual_norm(orc_h *H, const double *rho, const double *phi, const double *B) {
    orc_residual(H, 0, 2, phi, rho, B, H->r0);
    return norm2(H, 0, H->r0);
}

void orc_default_opts(orc_opts *o) {
    o->n_pre = 2; o->n_post = 2; o->n_cycles = 1; o->n_coarse = 32; o->max_cycles = 200;
    o->bc_order = 0; o->eta = 0.5; o->hold = 10;
}

/*
 * Solve loop (Sec. 2 "repeated until the residual is small enough"; Sec. 4
 * runtime order switch).  Status: 0 converged, 1 max_cycles reached,
 * -4 non-finite norm.  phi holds the initial guess on entry; inactive cells
 * of phi are never read or written.
 */
int orc_solve(orc_h *H, const double *rho, double *phi, const double *B, double tol, const orc_opts *o, orc_info *info) {
    orc_info tmp;
    if (!info) info = &tmp;
    memset(info, 0, sizeof(*info));
    info->switched_at = -1;
    /* reference: residual of phi = 0 */
    size_t n0 = ncell(H, 0);
    double *zero = (double *)calloc(n0, sizeof(double));
    double rref = orc_residual_norm(H, rho, zero, B);
    free(zero);
    double rprev = orc_residual_norm(H, rho, phi, B);
    info->r0 = rprev;
    if (rref == 0.0) rref = rprev;
    info->r_ref = rref;
    info->history[0] = rprev;
    int order;
    if (o->bc_order == 1 || o->bc_order == 2) order = o->bc_order;
    else if (H->hold_left > 0) { order = 1; H->hold_left--; }
    else order = 2;
    if (H->nlev[order] == 0) { info->status = -2; return -2; }
    info->order_used = order;
    info->r_final = rprev;
    if (!(rprev > tol * rref)) { info->status = 0; return 0; }
    for (int n = 1; n <= o->max_cycles; n++) {
        mg_level(H, 0, order, phi, rho, B, o);
        double rn = orc_residual_norm(H, rho, phi, B);
        info->cycles = n;
        info->r_final = rn;
        if (n < 257) info->history[n] = rn;
        if (!isfinite(rn)) { info->status = -4; return -4; }
        if (rn <= tol * rref) { info->status = 0; info->order_used = order; return 0; }
        if (o->bc_order == 0 && order == 2 && rn / rprev > o->eta) {
            order = 1;
            H->hold_left = o->hold;
            info->switched_at = n;
            info->order_used = 1;
        }
        rprev = rn;
    }
    info->status = 1;
    return 1;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
