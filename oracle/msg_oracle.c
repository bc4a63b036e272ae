/*
 * msg_oracle.c -- plain FP64 CPU oracle for batched Multiple Semi-Coarsened
 * Multigrid (MSG / full MSG) solves of the 2D lognormal diffusion problem and
 * the multi-index differences formed from their per-grid solutions.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no code, header, table or helper with the HIP path; the
 * two meet only in the documented array order (grids p-major then q-minor,
 * each grid row-major with x fastest) and in the seeded inputs.
 *
 * Everything is written the slow, literal way: one grid at a time, loops over
 * cells in row-major order, the operator applied face by face, weight factors
 * obtained by literally applying the operator to the two oscillating modes,
 * the coarsest grid solved through a dense Cholesky factorisation of the
 * matrix assembled column by column from the operator.
 *
 * Paper: Robbe, Nuyens, Vandewalle, "Enhanced Multi-Index Monte Carlo by
 * means of Multiple Semi-Coarsened Multigrid for Anisotropic Diffusion
 * Problems" (arXiv 1907.12334).  Citations below name the section, equation
 * or algorithm of that paper.
 *
 * Readings taken where the paper is silent or stated for a vertex-centred
 * finite-difference grid (the workload fixes a cell-centred finite-volume
 * grid); each is listed with its reason in the design notes:
 *   - grid (p,q) has nx = c*2^p by ny = c*2^q cells, hx = 1/nx, hy = 1/ny;
 *     index (0,0) is the coarsest c-by-c grid, level L = p + q;
 *   - the diffusion coefficient is evaluated at every face midpoint of
 *     every grid (direct discretisation on each grid, Section 2), or, under
 *     the face-mean rule, at the finest grid's face midpoints, every coarser
 *     face taking the mean of those lying on it (oracle_face_mean);
 *   - 5-point cell-centred finite volumes; a wall face carries twice the
 *     face conductance (half-cell distance to the Dirichlet wall, u = 0);
 *   - restriction in one direction averages the two fine cells covered by a
 *     coarse cell (the cell-centred analogue of full weighting);
 *   - prolongation in one direction is cell-centred linear interpolation
 *     (weights 3/4, 1/4) with odd reflection at the walls;
 *   - the nested-iteration interpolation is cell-centred cubic Lagrange
 *     interpolation (weights (-5,35,105,-7)/128 and mirror) with odd
 *     reflection at the walls, combined with the weight factors exactly as
 *     the coarse-grid correction is;
 *   - red cells are those with i + j even; a sweep is red then black;
 *   - the coarse-grid correction is multiplied by a damping factor omega
 *     (1 unless the caller chooses otherwise);
 *   - the adaptive cycle count checks ||r||_2 <= tol * ||b||_2 on every grid
 *     of the stage level before each cycle (zero cycles allowed);
 *   - the solution returned for grid (p,q) is the iterate at the end of
 *     stage p + q of the F-cycle, before later stages reuse the grid for
 *     corrections.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

/* per-sample status, mirrored by value in the public header of the product */
#define OR_CONVERGED 0
#define OR_MAXITER 1
#define OR_NONFINITE 2

/* ------------------------------------------------------------------------ */
/* One grid of the semi-coarsened hierarchy (Section 2, eq. hierarchy).      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int p, q;        /* grid index */
    int nx, ny;      /* number of cells in x and y */
    double hx, hy;   /* mesh widths */
    double *kx;      /* (nx+1)*ny coefficients on x-faces: face (i,j) at x=i*hx, y=(j+1/2)*hy */
    double *ky;      /* nx*(ny+1) coefficients on y-faces: face (i,j) at x=(i+1/2)*hx, y=j*hy */
    double *v;       /* iterate, nx*ny, index j*nx+i */
    double *b;       /* right-hand side, nx*ny */
    double *r;       /* residual scratch, nx*ny */
} ogrid;

typedef struct {
    int c, P, Q;     /* coarsest cells per direction, finest index (P,Q) */
    ogrid *g;        /* (P+1)*(Q+1) grids, index p*(Q+1)+q */
    double *chol;    /* Cholesky factor of the coarsest matrix, (c*c)^2 */
} ohier;

typedef struct {
    int32_t mu;          /* cycle index: 1 = V-cycle, 2 = W-cycle */
    int32_t nu1, nu2;    /* pre- and post-smoothing sweeps */
    int32_t max_cycles;  /* cap on cycles per F-cycle stage */
    double tol;          /* relative residual tolerance per grid */
    double omega;        /* damping of the coarse-grid correction */
    int32_t joint_stages; /* 1: cycle all grids of an F-cycle level together */
} oracle_opts;

static ogrid *grid_at(ohier *H, int p, int q) { return &H->g[p * (H->Q + 1) + q]; }
static int in_rect(const ohier *H, int p, int q) { return p >= 0 && q >= 0 && p <= H->P && q <= H->Q; }

/* ------------------------------------------------------------------------ */
/* Discrete operator: cell-centred 5-point finite volumes of -div(k grad u). */
/* ------------------------------------------------------------------------ */

/* conductance of x-face i (0..nx) in row j; wall faces are a half cell away */
static double cond_x(const ogrid *g, int i, int j)
{
    double wall = (i == 0 || i == g->nx) ? 2.0 : 1.0;
    return wall * g->kx[(size_t)j * (g->nx + 1) + i] / (g->hx * g->hx);
}

/* conductance of y-face j (0..ny) in column i */
static double cond_y(const ogrid *g, int i, int j)
{
    double wall = (j == 0 || j == g->ny) ? 2.0 : 1.0;
    return wall * g->ky[(size_t)j * g->nx + i] / (g->hy * g->hy);
}

/* value of u at cell (i,j), zero outside the domain (Dirichlet wall) */
static double at(const ogrid *g, const double *u, int i, int j)
{
    if (i < 0 || j < 0 || i >= g->nx || j >= g->ny) return 0.0;
    return u[(size_t)j * g->nx + i];
}

/* (A u)_ij: sum over the four faces of conductance times jump */
static double apply_cell(const ogrid *g, const double *u, int i, int j)
{
    double uc = at(g, u, i, j);
    return cond_x(g, i, j) * (uc - at(g, u, i - 1, j))
         + cond_x(g, i + 1, j) * (uc - at(g, u, i + 1, j))
         + cond_y(g, i, j) * (uc - at(g, u, i, j - 1))
         + cond_y(g, i, j + 1) * (uc - at(g, u, i, j + 1));
}

static void apply_grid(const ogrid *g, const double *u, double *out)
{
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i)
            out[(size_t)j * g->nx + i] = apply_cell(g, u, i, j);
}

/* r = b - A v on one grid */
static void residual_grid(const ogrid *g, const double *b, const double *v, double *r)
{
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i)
            r[(size_t)j * g->nx + i] = b[(size_t)j * g->nx + i] - apply_cell(g, v, i, j);
}

/* Red-black Gauss-Seidel, Section 2 (nu1 = nu2 = 2 sweeps of red then black) */
static void rbgs_sweep(const ogrid *g, const double *b, double *u)
{
    for (int colour = 0; colour < 2; ++colour)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                if (((i + j) & 1) != colour) continue;
                double wW = cond_x(g, i, j), wE = cond_x(g, i + 1, j);
                double wS = cond_y(g, i, j), wN = cond_y(g, i, j + 1);
                double num = b[(size_t)j * g->nx + i]
                           + wW * at(g, u, i - 1, j) + wE * at(g, u, i + 1, j)
                           + wS * at(g, u, i, j - 1) + wN * at(g, u, i, j + 1);
                u[(size_t)j * g->nx + i] = num / (wW + wE + wS + wN);
            }
}

/* ------------------------------------------------------------------------ */
/* Weight factors, eq. weight_factors: lambda_x = A f, lambda_y = A g with   */
/* f = cos(i pi), g = cos(j pi); kappa_x = lambda_x^2/(lambda_x^2+lambda_y^2) */
/* ------------------------------------------------------------------------ */
static void weights_grid(const ogrid *g, double *kap_x, double *kap_y)
{
    size_t n = (size_t)g->nx * g->ny;
    double *f = malloc(n * sizeof(double)), *gg = malloc(n * sizeof(double));
    double *lx = malloc(n * sizeof(double)), *ly = malloc(n * sizeof(double));
    for (int j = 0; j < g->ny; ++j)
        for (int i = 0; i < g->nx; ++i) {
            f[(size_t)j * g->nx + i] = cos(i * OR_PI);
            gg[(size_t)j * g->nx + i] = cos(j * OR_PI);
        }
    apply_grid(g, f, lx);
    apply_grid(g, gg, ly);
    for (size_t k = 0; k < n; ++k) {
        double a = lx[k] * lx[k], c = ly[k] * ly[k];
        kap_x[k] = a / (a + c);
        kap_y[k] = c / (a + c);
    }
    free(f); free(gg); free(lx); free(ly);
}

/* ------------------------------------------------------------------------ */
/* One-directional transfers (Section 2, restriction/prolongation operators) */
/* ------------------------------------------------------------------------ */

/* R_x: fine (2n_c x ny) -> coarse (n_c x ny), mean of the two covered cells */
static void restrict_x(int nxc, int ny, const double *fine, double *coarse)
{
    int nxf = 2 * nxc;
    for (int j = 0; j < ny; ++j)
        for (int I = 0; I < nxc; ++I)
            coarse[(size_t)j * nxc + I] = 0.5 * (fine[(size_t)j * nxf + 2 * I] + fine[(size_t)j * nxf + 2 * I + 1]);
}

/* R_y: fine (nx x 2n_c) -> coarse (nx x n_c) */
static void restrict_y(int nx, int nyc, const double *fine, double *coarse)
{
    for (int J = 0; J < nyc; ++J)
        for (int i = 0; i < nx; ++i)
            coarse[(size_t)J * nx + i] = 0.5 * (fine[(size_t)(2 * J) * nx + i] + fine[(size_t)(2 * J + 1) * nx + i]);
}

/* coarse value along one line with odd reflection at both walls */
static double odd_ext(const double *line, ptrdiff_t stride, int n, int I)
{
    if (I < 0) return -odd_ext(line, stride, n, -1 - I);
    if (I >= n) return -odd_ext(line, stride, n, 2 * n - 1 - I);
    return line[(ptrdiff_t)I * stride];
}

/* linear interpolation of one line of n coarse cells to 2n fine cells */
static void linear_line(const double *c, ptrdiff_t cs, int n, double *f, ptrdiff_t fs)
{
    for (int I = 0; I < n; ++I) {
        f[(ptrdiff_t)(2 * I) * fs] = 0.75 * odd_ext(c, cs, n, I) + 0.25 * odd_ext(c, cs, n, I - 1);
        f[(ptrdiff_t)(2 * I + 1) * fs] = 0.75 * odd_ext(c, cs, n, I) + 0.25 * odd_ext(c, cs, n, I + 1);
    }
}

/* cubic Lagrange interpolation of one line: the fine cell at I -/+ H/4 */
static void cubic_line(const double *c, ptrdiff_t cs, int n, double *f, ptrdiff_t fs)
{
    for (int I = 0; I < n; ++I) {
        f[(ptrdiff_t)(2 * I) * fs] = (-5.0 * odd_ext(c, cs, n, I - 2) + 35.0 * odd_ext(c, cs, n, I - 1)
                                      + 105.0 * odd_ext(c, cs, n, I) - 7.0 * odd_ext(c, cs, n, I + 1)) / 128.0;
        f[(ptrdiff_t)(2 * I + 1) * fs] = (-7.0 * odd_ext(c, cs, n, I - 1) + 105.0 * odd_ext(c, cs, n, I)
                                          + 35.0 * odd_ext(c, cs, n, I + 1) - 5.0 * odd_ext(c, cs, n, I + 2)) / 128.0;
    }
}

/* P_x: coarse (nxc x ny) -> fine (2nxc x ny); cubic selects the FMG stencil */
static void prolong_x(int nxc, int ny, const double *coarse, double *fine, int cubic)
{
    for (int j = 0; j < ny; ++j) {
        if (cubic) cubic_line(coarse + (size_t)j * nxc, 1, nxc, fine + (size_t)j * 2 * nxc, 1);
        else linear_line(coarse + (size_t)j * nxc, 1, nxc, fine + (size_t)j * 2 * nxc, 1);
    }
}

/* P_y: coarse (nx x nyc) -> fine (nx x 2nyc) */
static void prolong_y(int nx, int nyc, const double *coarse, double *fine, int cubic)
{
    for (int i = 0; i < nx; ++i) {
        if (cubic) cubic_line(coarse + i, nx, nyc, fine + i, nx);
        else linear_line(coarse + i, nx, nyc, fine + i, nx);
    }
}

/* ------------------------------------------------------------------------ */
/* Combination of the two semi-coarsened grids                               */
/* ------------------------------------------------------------------------ */

/* eq. restriction: b^(p,q) from the fine-grid quantity `which` (the residual
 * r inside a cycle, the right-hand side b in the F-cycle) of (p+1,q), (p,q+1) */
static void restrict_combine(ohier *H, int p, int q, int use_rhs)
{
    ogrid *g = grid_at(H, p, q);
    size_t n = (size_t)g->nx * g->ny;
    int hasx = in_rect(H, p + 1, q), hasy = in_rect(H, p, q + 1);
    double *tx = calloc(n, sizeof(double)), *ty = calloc(n, sizeof(double));
    if (hasx) {
        ogrid *f = grid_at(H, p + 1, q);
        restrict_x(g->nx, g->ny, use_rhs ? f->b : f->r, tx);
    }
    if (hasy) {
        ogrid *f = grid_at(H, p, q + 1);
        restrict_y(g->nx, g->ny, use_rhs ? f->b : f->r, ty);
    }
    for (size_t k = 0; k < n; ++k) {
        if (hasx && !hasy) g->b[k] = tx[k];             /* q = Q: only the x-coarsened parent */
        else if (hasy && !hasx) g->b[k] = ty[k];        /* p = P: only the y-coarsened parent */
        else g->b[k] = 0.5 * tx[k] + 0.5 * ty[k];       /* otherwise the average */
    }
    free(tx); free(ty);
}

/* eq. interpolation: the weighted combination of the interpolated coarse
 * iterates of (p-1,q) and (p,q-1) on grid (p,q); returned in `out` */
static void interp_combine(ohier *H, int p, int q, int cubic, double *out)
{
    ogrid *g = grid_at(H, p, q);
    size_t n = (size_t)g->nx * g->ny;
    int hasx = p > 0, hasy = q > 0;
    double *ex = calloc(n, sizeof(double)), *ey = calloc(n, sizeof(double));
    double *kx = malloc(n * sizeof(double)), *ky = malloc(n * sizeof(double));
    weights_grid(g, kx, ky);
    if (hasx) prolong_x(g->nx / 2, g->ny, grid_at(H, p - 1, q)->v, ex, cubic);
    if (hasy) prolong_y(g->nx, g->ny / 2, grid_at(H, p, q - 1)->v, ey, cubic);
    for (size_t k = 0; k < n; ++k) {
        if (hasx && !hasy) out[k] = ex[k];              /* q = 0: only P_x */
        else if (hasy && !hasx) out[k] = ey[k];         /* p = 0: only P_y */
        else out[k] = kx[k] * ex[k] + ky[k] * ey[k];
    }
    free(ex); free(ey); free(kx); free(ky);
}

/* ------------------------------------------------------------------------ */
/* Coarsest grid: dense Cholesky of A^(0,0), assembled column by column.      */
/* ------------------------------------------------------------------------ */
/* dense Cholesky factor L (n*n, n = nx*ny) of one grid's matrix */
static int dense_factor(const ogrid *g, double *L)
{
    int n = g->nx * g->ny;
    double *e = calloc((size_t)n, sizeof(double)), *col = malloc((size_t)n * sizeof(double));
    double *A = malloc((size_t)n * n * sizeof(double));
    for (int k = 0; k < n; ++k) {
        memset(e, 0, (size_t)n * sizeof(double));
        e[k] = 1.0;
        apply_grid(g, e, col);
        for (int m = 0; m < n; ++m) A[(size_t)m * n + k] = col[m];
    }
    memset(L, 0, (size_t)n * n * sizeof(double));
    int ok = 1;
    for (int j = 0; j < n; ++j) {
        double s = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(s > 0.0)) ok = 0;
        L[(size_t)j * n + j] = sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double t = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / L[(size_t)j * n + j];
        }
    }
    free(e); free(col); free(A);
    return ok;
}

/* v = A^{-1} b on one grid from its factor: forward then backward substitution */
static void dense_solve(ogrid *g, const double *L)
{
    int n = g->nx * g->ny;
    double *y = malloc((size_t)n * sizeof(double));
    for (int i = 0; i < n; ++i) {
        double s = g->b[i];
        for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * y[k];
        y[i] = s / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * g->v[k];
        g->v[i] = s / L[(size_t)i * n + i];
    }
    free(y);
}

static int coarse_factor(ohier *H) { return dense_factor(grid_at(H, 0, 0), H->chol); }

/* v^(0,0) = (A^(0,0))^{-1} b^(0,0) */
static void coarse_solve(ohier *H) { dense_solve(grid_at(H, 0, 0), H->chol); }

/* ------------------------------------------------------------------------ */
/* The mu-cycle (Algorithm 1 of Section 2) as a correction scheme over the   */
/* levels of the semi-coarsened family: a level is the set of grids (p,q)    */
/* with p + q = L inside the rectangle, and each operation below acts on all */
/* of them, one grid at a time.                                              */
/* ------------------------------------------------------------------------ */

/* the grids of level L, in order of increasing p; returns their count */
static int level_grids(const ohier *H, int L, int *ps)
{
    int n = 0;
    for (int p = 0; p <= H->P; ++p)
        if (in_rect(H, p, L - p)) ps[n++] = p;
    return n;
}

/* nu red-black sweeps on every grid of level L */
static void smooth_level(ohier *H, int L, int nu)
{
    int ps[64], n = level_grids(H, L, ps);
    for (int k = 0; k < n; ++k) {
        ogrid *g = grid_at(H, ps[k], L - ps[k]);
        for (int s = 0; s < nu; ++s) rbgs_sweep(g, g->b, g->v);
    }
}

/* the coarse problems of level L - 1: every grid of level L stores its
 * defect r = b - A v; every grid of level L - 1 takes the combination of its
 * parents' defects given by eq. restriction as right-hand side, and zero as
 * initial guess */
static void coarse_problems(ohier *H, int L)
{
    int ps[64], n = level_grids(H, L, ps);
    for (int k = 0; k < n; ++k) {
        ogrid *g = grid_at(H, ps[k], L - ps[k]);
        residual_grid(g, g->b, g->v, g->r);
    }
    n = level_grids(H, L - 1, ps);
    for (int k = 0; k < n; ++k) {
        ogrid *h = grid_at(H, ps[k], L - 1 - ps[k]);
        restrict_combine(H, ps[k], L - 1 - ps[k], 0);
        memset(h->v, 0, (size_t)h->nx * h->ny * sizeof(double));
    }
}

/* every grid of level L adds omega times the weighted interpolation of its
 * children's iterates (eq. interpolation with eq. weight_factors) */
static void correct_level(ohier *H, int L, double omega)
{
    int ps[64], n = level_grids(H, L, ps);
    for (int k = 0; k < n; ++k) {
        ogrid *g = grid_at(H, ps[k], L - ps[k]);
        size_t cells = (size_t)g->nx * g->ny;
        double *corr = malloc(cells * sizeof(double));
        interp_combine(H, ps[k], L - ps[k], 0, corr);
        for (size_t t = 0; t < cells; ++t) g->v[t] += omega * corr[t];
        free(corr);
    }
}

/* one mu-cycle on level L: the coarsest level is solved directly; above it,
 * pre-smoothing, mu cycles on the coarse problems, correction and
 * post-smoothing */
static void mu_cycle(ohier *H, int L, const oracle_opts *o)
{
    if (L == 0) {
        coarse_solve(H);
        return;
    }
    smooth_level(H, L, o->nu1);
    coarse_problems(H, L);
    for (int m = 0; m < o->mu; ++m) mu_cycle(H, L - 1, o);
    correct_level(H, L, o->omega);
    smooth_level(H, L, o->nu2);
}

static double norm2(const double *x, size_t n)
{
    double s = 0.0;
    for (size_t k = 0; k < n; ++k) s += x[k] * x[k];
    return sqrt(s);
}

/* ||b - A v||_2 / ||b||_2 on one grid; returns 1 if ||r|| <= tol ||b||,
 * -1 if a norm is not finite, else 0 */
static int grid_converged(ogrid *g, double tol, double *ratio)
{
    size_t n = (size_t)g->nx * g->ny;
    residual_grid(g, g->b, g->v, g->r);
    double rn = norm2(g->r, n), bn = norm2(g->b, n);
    if (!isfinite(rn) || !isfinite(bn)) { *ratio = NAN; return -1; }
    *ratio = bn > 0.0 ? rn / bn : (rn > 0.0 ? INFINITY : 0.0);
    return rn <= tol * bn;
}

/* ------------------------------------------------------------------------ */
/* Hierarchy set-up from packed per-grid face coefficients                   */
/* ------------------------------------------------------------------------ */
static void grid_geometry(ogrid *g, int c, int p, int q)
{
    g->p = p; g->q = q;
    g->nx = c << p; g->ny = c << q;
    g->hx = 1.0 / g->nx; g->hy = 1.0 / g->ny;
}

static void hier_init(ohier *H, int c, int P, int Q, const double *kx_all, const double *ky_all)
{
    H->c = c; H->P = P; H->Q = Q;
    H->g = calloc((size_t)(P + 1) * (Q + 1), sizeof(ogrid));
    size_t ox = 0, oy = 0;
    for (int p = 0; p <= P; ++p)
        for (int q = 0; q <= Q; ++q) {
            ogrid *g = grid_at(H, p, q);
            grid_geometry(g, c, p, q);
            size_t n = (size_t)g->nx * g->ny;
            size_t nfx = (size_t)(g->nx + 1) * g->ny, nfy = (size_t)g->nx * (g->ny + 1);
            g->kx = malloc(nfx * sizeof(double));
            g->ky = malloc(nfy * sizeof(double));
            memcpy(g->kx, kx_all + ox, nfx * sizeof(double));
            memcpy(g->ky, ky_all + oy, nfy * sizeof(double));
            ox += nfx; oy += nfy;
            g->v = calloc(n, sizeof(double));
            g->b = calloc(n, sizeof(double));
            g->r = calloc(n, sizeof(double));
        }
    H->chol = calloc((size_t)c * c * c * c, sizeof(double));
}

static void hier_free(ohier *H)
{
    for (int k = 0; k < (H->P + 1) * (H->Q + 1); ++k) {
        free(H->g[k].kx); free(H->g[k].ky); free(H->g[k].v); free(H->g[k].b); free(H->g[k].r);
    }
    free(H->g); free(H->chol);
}

/* The rectangle [0..p] x [0..q] below grid (p,q) of H, with (p,q) as its
 * finest grid: coefficients and the coarsest factor are those of H (shared,
 * read only); iterates, right-hand sides and residuals are its own. */
static void sub_init(ohier *S, ohier *H, int p, int q)
{
    S->c = H->c; S->P = p; S->Q = q;
    S->g = calloc((size_t)(p + 1) * (q + 1), sizeof(ogrid));
    for (int a = 0; a <= p; ++a)
        for (int s = 0; s <= q; ++s) {
            ogrid *g = grid_at(S, a, s);
            grid_geometry(g, H->c, a, s);
            size_t n = (size_t)g->nx * g->ny;
            g->kx = grid_at(H, a, s)->kx;
            g->ky = grid_at(H, a, s)->ky;
            g->v = calloc(n, sizeof(double));
            g->b = calloc(n, sizeof(double));
            g->r = calloc(n, sizeof(double));
        }
    S->chol = H->chol;
}

static void sub_free(ohier *S)
{
    for (int k = 0; k < (S->P + 1) * (S->Q + 1); ++k) {
        free(S->g[k].v); free(S->g[k].b); free(S->g[k].r);
    }
    free(S->g);
}

/* right-hand side on the finest grid: h = 1 at every cell centre, or given */
static void set_top_rhs(ohier *H, const double *rhs_top)
{
    ogrid *g = grid_at(H, H->P, H->Q);
    size_t n = (size_t)g->nx * g->ny;
    for (size_t k = 0; k < n; ++k) g->b[k] = rhs_top ? rhs_top[k] : 1.0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm MSG F-cycle (recursive definition) with adaptive nu0            */
/* ------------------------------------------------------------------------ */
typedef struct {
    const oracle_opts *o;
    const int32_t *forced;   /* NULL, or cycles per grid to run regardless of tol */
    int32_t *cycles;         /* cycles run per grid, [(P+1)(Q+1)] */
    double *hist;            /* NULL or [(P+1)(Q+1)][max_cycles+1] residual ratio per check */
    int status;
    int dead_level;          /* first level with a non-finite norm, or -1 */
} fctx;

/* Adaptive nu0 on one grid of level L: mu-cycles over its own rectangle
 * until ||r|| <= tol ||b|| (checked before every cycle, zero cycles allowed) */
static void solve_grid(ohier *H, int p, int q, fctx *F)
{
    const oracle_opts *o = F->o;
    int gi = p * (H->Q + 1) + q, hc = o->max_cycles + 1;
    ogrid *top = grid_at(H, p, q);
    size_t n = (size_t)top->nx * top->ny;
    ohier S;
    sub_init(&S, H, p, q);
    ogrid *st = grid_at(&S, p, q);
    memcpy(st->v, top->v, n * sizeof(double));
    memcpy(st->b, top->b, n * sizeof(double));
    int ncyc = 0;
    for (;;) {
        double ratio;
        int conv = grid_converged(st, o->tol, &ratio);
        if (F->hist && ncyc < hc) F->hist[(size_t)gi * hc + ncyc] = ratio;
        if (conv < 0) { F->status = OR_NONFINITE; F->dead_level = p + q; break; }
        if (F->forced) {
            if (ncyc >= F->forced[gi]) break;
        } else {
            if (conv) break;
            if (ncyc >= o->max_cycles) { if (F->status == OR_CONVERGED) F->status = OR_MAXITER; break; }
        }
        mu_cycle(&S, p + q, o);
        ++ncyc;
    }
    F->cycles[gi] = ncyc;
    memcpy(top->v, st->v, n * sizeof(double));
    sub_free(&S);
}

/* the literal alternative: all grids of level L cycle together in the full
 * rectangle, sharing (and averaging into) the coarse grids below them */
static void solve_level_joint(ohier *H, int L, fctx *F)
{
    const oracle_opts *o = F->o;
    int hc = o->max_cycles + 1, ncyc = 0;
    for (;;) {
        int all = 1, bad = 0;
        for (int p = 0; p <= H->P; ++p) {
            int q = L - p;
            if (!in_rect(H, p, q)) continue;
            double ratio;
            int conv = grid_converged(grid_at(H, p, q), o->tol, &ratio);
            if (F->hist && ncyc < hc) F->hist[(size_t)(p * (H->Q + 1) + q) * hc + ncyc] = ratio;
            if (conv < 0) bad = 1;
            if (conv != 1) all = 0;
        }
        if (bad) { F->status = OR_NONFINITE; F->dead_level = L; break; }
        if (F->forced) {
            int p0 = L > H->Q ? L - H->Q : 0;     /* first grid of level L sets the count */
            if (ncyc >= F->forced[p0 * (H->Q + 1) + L - p0]) break;
        } else {
            if (all) break;
            if (ncyc >= o->max_cycles) { if (F->status == OR_CONVERGED) F->status = OR_MAXITER; break; }
        }
        mu_cycle(H, L, o);
        ++ncyc;
    }
    for (int p = 0; p <= H->P; ++p)
        if (in_rect(H, p, L - p)) F->cycles[p * (H->Q + 1) + L - p] = ncyc;
}

static void f_cycle(ohier *H, int L, fctx *F)
{
    if (L == 0) {
        memset(grid_at(H, 0, 0)->v, 0, (size_t)H->c * H->c * sizeof(double));
    } else {
        for (int p = 0; p <= H->P; ++p) {               /* restrict the right-hand side to L-1 */
            int q = L - 1 - p;
            if (in_rect(H, p, q)) restrict_combine(H, p, q, 1);
        }
        f_cycle(H, L - 1, F);
        if (F->dead_level >= 0) return;
        for (int p = 0; p <= H->P; ++p) {               /* interpolated solution on level L */
            int q = L - p;
            if (!in_rect(H, p, q)) continue;
            interp_combine(H, p, q, 1, grid_at(H, p, q)->v);
        }
    }
    if (F->o->joint_stages) {
        solve_level_joint(H, L, F);
    } else {
        for (int p = 0; p <= H->P; ++p)
            if (in_rect(H, p, L - p)) solve_grid(H, p, L - p, F);
    }
}

/* ======================================================================== */
/* Exported entry points (ctypes)                                           */
/* ======================================================================== */

/* Full MSG solve of one sample (Algorithm MSG F-cycle with the mu-cycle).
 * kx_all / ky_all: face coefficients of every grid, packed p-major, q-minor.
 * rhs_top: NULL for h = 1, else nx*ny values on the finest grid.
 * forced_cycles: NULL for the adaptive rule, else cycles to run per grid.
 * u_out: every grid's returned solution, packed like the cells.
 * q_out: (P+1)*(Q+1) means of u.  cycles_out: cycles per grid.
 * hist: NULL or (P+1)*(Q+1)*(max_cycles+1) residual ratios per check.
 * Returns the sample status (0 converged, 1 cycle cap hit, 2 non-finite);
 * after a non-finite norm on level L, grids of levels >= L hold NaN. */
int oracle_fmsg_solve(int c, int P, int Q, const double *kx_all, const double *ky_all,
                      const double *rhs_top, const oracle_opts *o, const int32_t *forced_cycles,
                      double *u_out, double *q_out, int32_t *cycles_out, double *hist)
{
    ohier H;
    hier_init(&H, c, P, Q, kx_all, ky_all);
    set_top_rhs(&H, rhs_top);
    fctx F = { o, forced_cycles, cycles_out, hist, OR_CONVERGED, -1 };
    for (int k = 0; k < (P + 1) * (Q + 1); ++k) cycles_out[k] = 0;
    if (!coarse_factor(&H)) {
        F.status = OR_NONFINITE;
        F.dead_level = 0;
    } else {
        f_cycle(&H, P + Q, &F);
    }
    size_t off = 0;
    for (int p = 0; p <= P; ++p)
        for (int q = 0; q <= Q; ++q) {
            ogrid *g = grid_at(&H, p, q);
            size_t n = (size_t)g->nx * g->ny;
            int dead = F.dead_level >= 0 && p + q >= F.dead_level;
            double s = 0.0;
            for (size_t k = 0; k < n; ++k) {
                u_out[off + k] = dead ? NAN : g->v[k];
                s += g->v[k];
            }
            q_out[p * (Q + 1) + q] = dead ? NAN : s / (double)n;   /* mean of u (midpoint rule) */
            off += n;
        }
    hier_free(&H);
    return F.status;
}

/* Plain MSG iteration on the finest grid (Algorithm MSG mu-cycle started
 * from v = 0 on level P+Q), ncycles cycles; u_top receives the iterate and
 * ratios[k] = ||r_k|| / ||b|| before cycle k (k = 0..ncycles). */
void oracle_msg_cycles(int c, int P, int Q, const double *kx_all, const double *ky_all,
                       const double *rhs_top, const oracle_opts *o, int ncycles,
                       double *u_top, double *ratios)
{
    ohier H;
    hier_init(&H, c, P, Q, kx_all, ky_all);
    set_top_rhs(&H, rhs_top);
    coarse_factor(&H);
    ogrid *g = grid_at(&H, P, Q);
    size_t n = (size_t)g->nx * g->ny;
    double bn = norm2(g->b, n);
    for (int k = 0; k <= ncycles; ++k) {
        residual_grid(g, g->b, g->v, g->r);
        ratios[k] = norm2(g->r, n) / bn;
        if (k < ncycles) mu_cycle(&H, P + Q, o);
    }
    memcpy(u_top, g->v, n * sizeof(double));
    hier_free(&H);
}

/* ------------------------------------------------------------------------ */
/* Standard-coarsening multigrid, the comparison of Section 2 (its Fig. of    */
/* convergence factors): grid (p,q) coarsens to (p-1,q-1) until one index is */
/* zero, where the grid is solved directly.  Restriction and prolongation are */
/* the products of the one-directional cell-centred operators (the 2D average */
/* of four cells, and bilinear interpolation), the operator is rediscretised */
/* on every grid, the smoother is the same red-black Gauss-Seidel.            */
/* ------------------------------------------------------------------------ */
static void mg_cycle(ohier *H, int k, int m, const double *Lc, const oracle_opts *o)
{
    ogrid *g = grid_at(H, H->P - k, H->Q - k);
    if (k == m) { dense_solve(g, Lc); return; }
    ogrid *gc = grid_at(H, H->P - k - 1, H->Q - k - 1);
    size_t n = (size_t)g->nx * g->ny;
    for (int s = 0; s < o->nu1; ++s) rbgs_sweep(g, g->b, g->v);
    residual_grid(g, g->b, g->v, g->r);
    double *half = malloc((size_t)gc->nx * g->ny * sizeof(double));
    restrict_x(gc->nx, g->ny, g->r, half);               /* (nx, ny) -> (nx/2, ny) */
    restrict_y(gc->nx, gc->ny, half, gc->b);             /* -> (nx/2, ny/2) */
    memset(gc->v, 0, (size_t)gc->nx * gc->ny * sizeof(double));
    for (int t = 0; t < o->mu; ++t) mg_cycle(H, k + 1, m, Lc, o);
    double *corr = malloc(n * sizeof(double));
    prolong_y(gc->nx, gc->ny, gc->v, half, 0);           /* (nx/2, ny/2) -> (nx/2, ny) */
    prolong_x(gc->nx, g->ny, half, corr, 0);             /* -> (nx, ny) */
    for (size_t t = 0; t < n; ++t) g->v[t] += o->omega * corr[t];
    for (int s = 0; s < o->nu2; ++s) rbgs_sweep(g, g->b, g->v);
    free(half); free(corr);
}

/* ncycles standard-multigrid mu-cycles from zero on the finest grid (P,Q);
 * ratios[k] = ||b - A v_k|| / ||b|| for k = 0..ncycles. */
void oracle_mg_cycles(int c, int P, int Q, const double *kx_all, const double *ky_all,
                      const double *rhs_top, const oracle_opts *o, int ncycles,
                      double *u_top, double *ratios)
{
    ohier H;
    hier_init(&H, c, P, Q, kx_all, ky_all);
    set_top_rhs(&H, rhs_top);
    const int m = P < Q ? P : Q;
    ogrid *gm = grid_at(&H, P - m, Q - m);
    size_t nm = (size_t)gm->nx * gm->ny;
    double *Lc = malloc(nm * nm * sizeof(double));
    dense_factor(gm, Lc);
    ogrid *g = grid_at(&H, P, Q);
    size_t n = (size_t)g->nx * g->ny;
    double bn = norm2(g->b, n);
    for (int k = 0; k <= ncycles; ++k) {
        residual_grid(g, g->b, g->v, g->r);
        ratios[k] = norm2(g->r, n) / bn;
        if (k < ncycles) mg_cycle(&H, 0, m, Lc, o);
    }
    memcpy(u_top, g->v, n * sizeof(double));
    free(Lc);
    hier_free(&H);
}

/* Multi-index difference (Section 3): Delta Q_l = (Delta_1 x Delta_2) Q_l
 * with Delta_i Q_l = Q_l - Q_{l-e_i} if l_i > 0, else Q_l. */
void oracle_delta_q(int P, int Q, const double *q, double *dq)
{
    for (int p = 0; p <= P; ++p)
        for (int s = 0; s <= Q; ++s) {
            double d = q[p * (Q + 1) + s];
            if (p > 0) d -= q[(p - 1) * (Q + 1) + s];
            if (s > 0) d -= q[p * (Q + 1) + s - 1];
            if (p > 0 && s > 0) d += q[(p - 1) * (Q + 1) + s - 1];
            dq[p * (Q + 1) + s] = d;
        }
}

/* Quantities of interest of Section 5 on one grid, from its cell values u
 * (row-major, x fastest) and, for the flux, its x-face coefficients kx
 * ((nx+1) per row).  Readings for the cell-centred grid:
 *   kind 0: mean of u over the cells (the workload's QoI, midpoint rule);
 *   kind 1: u at (1/2, 1/2), the bilinear interpolant of the cell-centre
 *           values (the point is a cell centre or lies between centres);
 *   kind 2: the average over D_sub = [1/4,1/2]^2 of the piecewise-constant
 *           finite-volume solution: each cell weighted by its overlap with
 *           D_sub (exact for that reconstruction at any alignment);
 *   kind 3: the flux -int_0^1 k du/dx dy through the wall x = 1: per row,
 *           the wall face's flux 2 k u / h_x (one-sided difference over the
 *           half cell to u = 0) times the face length h_y. */
double oracle_qoi_grid(int nx, int ny, const double *kx, const double *u, int kind)
{
    if (kind == 0) {
        double s = 0.0;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) s += u[j * nx + i];
        return s / ((double)nx * ny);
    }
    if (kind == 1) {
        /* fractional cell index of x = 1/2: centres sit at (i + 1/2)/n */
        const double tx = 0.5 * nx - 0.5, ty = 0.5 * ny - 0.5;
        const int i0 = (int)floor(tx), j0 = (int)floor(ty);
        const double wx = tx - i0, wy = ty - j0;
        double val = 0.0;
        for (int dj = 0; dj <= 1; ++dj)
            for (int di = 0; di <= 1; ++di) {
                const double w = (di ? wx : 1.0 - wx) * (dj ? wy : 1.0 - wy);
                if (w == 0.0) continue;
                val += w * u[(j0 + dj) * nx + (i0 + di)];
            }
        return val;
    }
    if (kind == 2) {
        const double lo = 0.25, hi = 0.5;
        double s = 0.0;
        for (int j = 0; j < ny; ++j) {
            const double oy = fmin((j + 1.0) / ny, hi) - fmax((double)j / ny, lo);
            if (oy <= 0.0) continue;
            for (int i = 0; i < nx; ++i) {
                const double ox = fmin((i + 1.0) / nx, hi) - fmax((double)i / nx, lo);
                if (ox <= 0.0) continue;
                s += u[j * nx + i] * ox * oy;
            }
        }
        return s / ((hi - lo) * (hi - lo));
    }
    /* kind 3 */
    const double hx = 1.0 / nx, hy = 1.0 / ny;
    double s = 0.0;
    for (int j = 0; j < ny; ++j) {
        const double k = kx[j * (nx + 1) + nx];
        s += 2.0 * k * (u[j * nx + nx - 1] - 0.0) / hx * hy;
    }
    return s;
}

/* ---- single-grid steps, exported so tests can pin each one ------------- */

static ogrid make_view(int nx, int ny, const double *kx, const double *ky)
{
    ogrid g;
    memset(&g, 0, sizeof g);
    g.nx = nx; g.ny = ny; g.hx = 1.0 / nx; g.hy = 1.0 / ny;
    g.kx = (double *)kx; g.ky = (double *)ky;
    return g;
}

void oracle_apply(int nx, int ny, const double *kx, const double *ky, const double *u, double *out)
{
    ogrid g = make_view(nx, ny, kx, ky);
    apply_grid(&g, u, out);
}

void oracle_residual(int nx, int ny, const double *kx, const double *ky, const double *b,
                     const double *u, double *r)
{
    ogrid g = make_view(nx, ny, kx, ky);
    residual_grid(&g, b, u, r);
}

void oracle_rbgs(int nx, int ny, const double *kx, const double *ky, const double *b, double *u, int sweeps)
{
    ogrid g = make_view(nx, ny, kx, ky);
    for (int s = 0; s < sweeps; ++s) rbgs_sweep(&g, b, u);
}

void oracle_weights(int nx, int ny, const double *kx, const double *ky, double *kap_x, double *kap_y)
{
    ogrid g = make_view(nx, ny, kx, ky);
    weights_grid(&g, kap_x, kap_y);
}

void oracle_restrict_x(int nxc, int ny, const double *fine, double *coarse) { restrict_x(nxc, ny, fine, coarse); }
void oracle_restrict_y(int nx, int nyc, const double *fine, double *coarse) { restrict_y(nx, nyc, fine, coarse); }
void oracle_prolong_x(int nxc, int ny, const double *coarse, double *fine, int cubic) { prolong_x(nxc, ny, coarse, fine, cubic); }
void oracle_prolong_y(int nx, int nyc, const double *coarse, double *fine, int cubic) { prolong_y(nx, nyc, coarse, fine, cubic); }

/* The combined interpolation of eq. interpolation on grid (p,q) alone: e_x
 * lives on (p-1,q) and e_y on (p,q-1) (either may be NULL when that grid does
 * not exist, p = 0 or q = 0); kx, ky are the face coefficients of (p,q);
 * cubic selects the nested-iteration stencil instead of linear. */
void oracle_correction(int c, int p, int q, const double *kx, const double *ky,
                       const double *e_x, const double *e_y, int cubic, double *out)
{
    ohier H;
    H.c = c; H.P = p; H.Q = q; H.chol = NULL;
    H.g = calloc((size_t)(p + 1) * (q + 1), sizeof(ogrid));
    ogrid *f = grid_at(&H, p, q);
    grid_geometry(f, c, p, q);
    f->kx = (double *)kx; f->ky = (double *)ky;
    if (p > 0) { grid_geometry(grid_at(&H, p - 1, q), c, p - 1, q); grid_at(&H, p - 1, q)->v = (double *)e_x; }
    if (q > 0) { grid_geometry(grid_at(&H, p, q - 1), c, p, q - 1); grid_at(&H, p, q - 1)->v = (double *)e_y; }
    interp_combine(&H, p, q, cubic, out);
    free(H.g);
}

/* ======================================================================== */
/* Random coefficient fields k = exp(Z) evaluated at face midpoints         */
/* ======================================================================== */

/* Z(x,y) = sum_t amp_t xi_t cos(pi a_t x) cos(pi b_t y) (cosine KL sum) */
static double z_cos(double x, double y, int nterms, const int32_t *a, const int32_t *b,
                    const double *amp, const double *xi)
{
    double z = 0.0;
    for (int t = 0; t < nterms; ++t)
        z += amp[t] * xi[t] * cos(OR_PI * a[t] * x) * cos(OR_PI * b[t] * y);
    return z;
}

void oracle_field_cos(int nx, int ny, int nterms, const int32_t *a, const int32_t *b,
                      const double *amp, const double *xi, double *kx, double *ky)
{
    double hx = 1.0 / nx, hy = 1.0 / ny;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i <= nx; ++i)
            kx[(size_t)j * (nx + 1) + i] = exp(z_cos(i * hx, (j + 0.5) * hy, nterms, a, b, amp, xi));
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i < nx; ++i)
            ky[(size_t)j * nx + i] = exp(z_cos((i + 0.5) * hx, j * hy, nterms, a, b, amp, xi));
}

/* separable squared-exponential KL: 1-D eigenpairs per direction,
 * phi_0 = 1, phi_k = sqrt(2) cos(pi k x), lambda_k proportional to
 * exp(-pi^2 l^2 k^2 / 2) and normalised to sum 1, so the domain-averaged
 * variance of Z is sigma^2; xi index m*my + n pairs x-mode m with y-mode n */
static void se_eigs(int m, double l, double *lam)
{
    double s = 0.0;
    for (int k = 0; k < m; ++k) { lam[k] = exp(-OR_PI * OR_PI * l * l * k * k / 2.0); s += lam[k]; }
    for (int k = 0; k < m; ++k) lam[k] /= s;
}

static double phi(int k, double x) { return k == 0 ? 1.0 : sqrt(2.0) * cos(OR_PI * k * x); }

/* Z at one point: the double sum over (m,n) of the definition; the basis
 * values at this point are tabulated first so each is computed once */
static double z_sep(double x, double y, int mx, int my, const double *amp, double sigma,
                    const double *xi, double *px, double *py)
{
    for (int m = 0; m < mx; ++m) px[m] = phi(m, x);
    for (int n = 0; n < my; ++n) py[n] = phi(n, y);
    double z = 0.0;
    for (int m = 0; m < mx; ++m)
        for (int n = 0; n < my; ++n)
            z += amp[m * my + n] * xi[m * my + n] * px[m] * py[n];
    return sigma * z;
}

/* Face-mean coefficients of grid (p,q) of a sample whose finest grid is
 * (P,Q) (reading R2b; direct discretisation on every grid, Section 2, with
 * the face flux taken as the mean of k along the face).  An x-face of grid
 * (p,q) lies on the line x = i/nx, which is also an x-face line of the
 * finest grid, and spans m = 2^(Q-q) rows of the finest grid; its
 * coefficient is the plain mean of k at the midpoints of those m finest
 * x-faces (midpoint rule for the mean of k along the face).  Likewise a
 * y-face spans 2^(P-p) columns of finest y-faces.  kxF, kyF: the finest
 * grid's pointwise face values; kx, ky: grid (p,q)'s faces (outputs). */
void oracle_face_mean(int c, int P, int Q, const double *kxF, const double *kyF, int p, int q,
                      double *kx, double *ky)
{
    int nxF = c << P, nx = c << p, ny = c << q;
    int rx = 1 << (P - p), ry = 1 << (Q - q);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            double s = 0.0;
            for (int t = 0; t < ry; ++t) s += kxF[(size_t)(j * ry + t) * (nxF + 1) + (size_t)i * rx];
            kx[(size_t)j * (nx + 1) + i] = s / ry;
        }
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double s = 0.0;
            for (int t = 0; t < rx; ++t) s += kyF[(size_t)j * ry * nxF + (size_t)i * rx + t];
            ky[(size_t)j * nx + i] = s / rx;
        }
}

void oracle_field_separable(int nx, int ny, int mx, int my, double lenx, double leny, double sigma2,
                            const double *xi, double *kx, double *ky)
{
    double hx = 1.0 / nx, hy = 1.0 / ny, sigma = sqrt(sigma2);
    double *lx = malloc((size_t)mx * sizeof(double)), *ly = malloc((size_t)my * sizeof(double));
    double *amp = malloc((size_t)mx * my * sizeof(double));
    double *px = malloc((size_t)mx * sizeof(double)), *py = malloc((size_t)my * sizeof(double));
    se_eigs(mx, lenx, lx);
    se_eigs(my, leny, ly);
    for (int m = 0; m < mx; ++m)
        for (int n = 0; n < my; ++n) amp[m * my + n] = sqrt(lx[m] * ly[n]);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i <= nx; ++i)
            kx[(size_t)j * (nx + 1) + i] = exp(z_sep(i * hx, (j + 0.5) * hy, mx, my, amp, sigma, xi, px, py));
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i < nx; ++i)
            ky[(size_t)j * nx + i] = exp(z_sep((i + 0.5) * hx, j * hy, mx, my, amp, sigma, xi, px, py));
    free(lx); free(ly); free(amp); free(px); free(py);
}
