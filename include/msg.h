/*
 * msg.h -- C-ABI of the MI355X batched Multiple Semi-Coarsened Multigrid
 * (MSG) library: lognormal coefficient fields, batched full-MSG solves that
 * return the solution on every semi-coarsened grid, and the multi-index
 * differences of the per-grid quantities of interest.
 *
 * Paper: Robbe, Nuyens, Vandewalle, "Enhanced Multi-Index Monte Carlo by
 * means of Multiple Semi-Coarsened Multigrid for Anisotropic Diffusion
 * Problems" (arXiv 1907.12334).
 *
 * Problem (Section 1, eq. PDE): -div(k grad u) = h on the unit square,
 * u = 0 on its boundary, k = exp(Z) with Z a Gaussian random field.
 *
 * Grids (Section 2, eq. hierarchy): a sample with finest index (P,Q) owns the
 * rectangle of grids (p,q), 0 <= p <= P, 0 <= q <= Q; grid (p,q) has
 * nx = c*2^p by ny = c*2^q cells (cell-centred finite volumes, mesh widths
 * 1/nx and 1/ny), c being the coarsest number of cells per direction.
 *
 * Layout (the single convention shared by every array of this header):
 *   - samples are packed one after another in batch order;
 *   - inside a sample, grids are packed p-major then q-minor;
 *   - inside a grid, values are row-major with x fastest:
 *       cells   nx*ny        index j*nx + i,      cell centre ((i+1/2)/nx, (j+1/2)/ny)
 *       x-faces (nx+1)*ny    index j*(nx+1) + i,  face at (i/nx, (j+1/2)/ny)
 *       y-faces nx*(ny+1)    index j*nx + i,      face at ((i+1/2)/nx, j/ny)
 *   - per-grid scalars (Q, Delta Q, cycle counts) are packed the same way,
 *     (P+1)*(Q+1) per sample.
 * msg_layout() returns every offset; it is the source of truth.
 *
 * Conventions: "d_" pointers are device pointers (HIP global memory on the
 * handle's device), owned by the caller; the library never frees them and
 * keeps no reference after a call returns.  Host arrays are read during the
 * call only.  Every call reports argument and layout errors through its
 * return value before touching the device; msg_last_error() then holds a
 * message (thread-local, valid until the next call on that thread).  Calls
 * are not re-entrant on one handle.
 */
#ifndef MSG_H
#define MSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct msg_handle_s *msg_handle;
typedef void *msg_stream;   /* a hipStream_t; NULL is the null stream */

typedef enum {
    MSG_OK = 0,
    MSG_ERR_ARG = -1,          /* bad argument (NULL, size, option out of range) */
    MSG_ERR_LAYOUT = -2,       /* batch shape outside the supported range */
    MSG_ERR_WORKSPACE = -3,    /* workspace smaller than msg_workspace_size() */
    MSG_ERR_HIP = -4,          /* a HIP runtime call failed */
    MSG_ERR_UNSUPPORTED = -5   /* combination of options not implemented */
} msg_status;

/* per-sample outcome written to d_status */
enum { MSG_SAMPLE_CONVERGED = 0, MSG_SAMPLE_MAXITER = 1, MSG_SAMPLE_NONFINITE = 2 };

/* field kinds (Section 1: k = exp(Z), Z Gaussian) */
enum {
    /* Z(x,y) = sum_t amp_t xi_t cos(pi a_t x) cos(pi b_t y), t < n_terms */
    MSG_FIELD_COS_TABLE = 0,
    /* separable squared-exponential Karhunen-Loeve expansion: per direction
     * phi_0 = 1, phi_k = sqrt(2) cos(pi k x), eigenvalues proportional to
     * exp(-pi^2 l^2 k^2 / 2) normalised to sum one, and
     * Z = sqrt(sigma2) sum_{m<mx, n<my} sqrt(lam_m lam_n) xi_{m*my+n} phi_m(x) phi_n(y) */
    MSG_FIELD_SEPARABLE_SE = 1
};

enum { MSG_FP64 = 0, MSG_MIXED = 1 };

/* How k enters the face conductances of each grid (direct discretisation
 * on every grid, Section 2; the paper does not say where k is sampled):
 *   MSG_FACE_POINT  k at the midpoint of every face of every grid;
 *   MSG_FACE_MEAN   k at the midpoints of the finest grid's faces, and on
 *                   every coarser grid the plain mean of the finest-grid
 *                   values along each face: an x-face of grid (p,q) lies on
 *                   an x-face line of the finest grid (P,Q) and spans 2^(Q-q)
 *                   of its faces; a y-face spans 2^(P-p) finest y-faces.
 *                   The coarse operators are then those of the mean flux
 *                   through each face, which keeps them consistent with the
 *                   finer grids when k varies below the coarse mesh width.
 *                   A grid's coefficients depend on the sample's finest
 *                   grid, so samples whose differences are combined in one
 *                   estimator must share their finest grid. */
enum { MSG_FACE_POINT = 0, MSG_FACE_MEAN = 1 };

typedef struct {
    int32_t kind;               /* MSG_FIELD_* */
    int32_t n_terms;            /* COS_TABLE: number of terms; SEPARABLE_SE: mx*my */
    const int32_t *a;           /* COS_TABLE: host [n_terms] x-frequencies (>= 0) */
    const int32_t *b;           /* COS_TABLE: host [n_terms] y-frequencies (>= 0) */
    const double *amp;          /* COS_TABLE: host [n_terms] amplitudes */
    int32_t mx, my;             /* SEPARABLE_SE: modes per direction */
    double lx, ly, sigma2;      /* SEPARABLE_SE: correlation lengths and variance */
    int32_t face_rule;          /* MSG_FACE_POINT or MSG_FACE_MEAN */
    int32_t reserved;           /* 0 */
    /* Used when msg_sample_field gets d_xi = NULL: the standard normals are
     * drawn on the device, xi[t] of a sample being normal t of the stream
     * (seed, sample id): Philox4x64-10 (Salmon et al. 2011) at counter
     * (t / 4, sample id, 0, 0) with key (seed, 0x4B4C2D7869), whose four
     * words w give u = ((w >> 12) + 1/2) 2^-52 and, by the Box-Muller
     * transform of words (0,1) and (2,3), the normals t = 4n, 4n+1 (cosine,
     * sine of the first pair) and 4n+2, 4n+3 (of the second pair). */
    uint64_t seed;
    const int64_t *sample_id;   /* host [n_samples], or NULL for 0..n_samples-1 */
} msg_field_spec;

typedef struct {
    int32_t n_samples;          /* S >= 1 */
    int32_t c;                  /* coarsest cells per direction, 1..8 */
    const int32_t *P;           /* host [S] finest x index, 0..14 */
    const int32_t *Q;           /* host [S] finest y index, 0..14 */
} msg_batch_desc;

typedef struct {
    int32_t mu;                 /* 1 = V-cycle, 2 = W-cycle (Section 2) */
    int32_t nu1, nu2;           /* red-black Gauss-Seidel sweeps before / after */
    int32_t max_cycles;         /* cap on cycles per grid of the F-cycle */
    double tol;                 /* stop when ||b - A v||_2 <= tol ||b||_2 per grid */
    double omega;               /* damping of the coarse-grid correction (1 = none) */
    int32_t precision;          /* MSG_FP64, or MSG_MIXED: FP32 inner cycles refined in FP64 */
    int32_t tail_levels;        /* -1 = automatic; else levels 0..tail_levels run in one
                                   workgroup per grid from on-chip memory */
    int32_t handoff;            /* -1 = automatic; 0 = never; n: once at most n problems of a
                                   class still cycle and its rectangle fits on chip, their
                                   remaining cycles run inside one kernel */
    int32_t overlap;            /* -1 = automatic (2 for 1024 samples or more, else 0);
                                   0 = every launch on `stream`; 1 = the cycles of the classes
                                   of a level alternate over side streams (four; environment
                                   MSG_SIDE_STREAMS = 1..4) forked from and joined back to
                                   `stream`; 2 = the batch is split in parts
                                   (three by default; environment MSG_PARTS = 2..4) solved
                                   concurrently by one host thread each, each part on one
                                   stream of its own.  Results do not depend on it; the
                                   workspace size does (msg_workspace_size). */
    /* Plan tuning (0 = the library's defaults; see paper_1907_12334_amd/autotune.py).
     * None changes results beyond rounding; all change the workspace size. */
    int32_t tail_budget;        /* LDS bytes per problem of the on-chip cycle tail (sets its
                                   depth): 0 or 1024..153600; default 20480, set for
                                   thousands of resident problems.  Above 40960 the tail runs
                                   on four wavefronts, and rectangles within the budget are
                                   solved whole in one kernel: for batches of few large
                                   samples, where each level kept on chip halves the host
                                   level visits of a cycle */
    int32_t tile_width;         /* smoother tile width cap: 0 or a power of two 4..256; default 64 */
    int32_t tile_cells;         /* smoother tile cell cap: 0 or 64..4096; default 1024 */
    int32_t tile_lds;           /* smoother tile LDS elements with halo: 0 or 256..8192;
                                   default 2048 */
    int32_t graphs;             /* 1 = capture each class's W-cycle as a HIP graph on its first
                                   cycle of a stage and replay it for the others (not while
                                   kernel timing is on); 0 = launch every kernel (default) */
} msg_solve_opts;

/* Fill opts with the defaults: W(2,2), 50 cycles, tol 1e-10, omega 1, FP64,
 * automatic tail depth, handoff and overlap. */
void msg_default_opts(msg_solve_opts *opts);

/* Create a handle bound to HIP device `device`.  Returns MSG_OK or MSG_ERR_HIP. */
msg_status msg_create(msg_handle *h, int device);
void msg_destroy(msg_handle h);
const char *msg_last_error(void);

/* Offsets of the packed layout.  All outputs are host arrays the caller
 * sizes: cell_off, xface_off, yface_off have n_samples+1 entries (sample
 * starts, last = totals); grid_off has n_samples+1 entries indexing the
 * per-grid scalar arrays.  Any output pointer may be NULL. */
msg_status msg_layout(const msg_batch_desc *batch, int64_t *cell_off, int64_t *xface_off,
                      int64_t *yface_off, int64_t *grid_off);

/* Bytes of device workspace msg_solve_batch needs for this batch and options. */
msg_status msg_workspace_size(msg_handle h, const msg_batch_desc *batch,
                              const msg_solve_opts *opts, size_t *bytes);

/* Coefficient field k = exp(Z) on the faces of every grid of every sample
 * (direct discretisation on each grid, Section 2; the paper samples Z
 * exactly, Section 5 -- here Z is the KL sum of msg_field_spec, and
 * spec->face_rule says where k is taken on each face).
 * d_xi: device [S][n_terms] standard normal coefficients, row per sample, or
 * NULL to draw them on the device from spec->seed and spec->sample_id.
 * d_kx, d_ky: device FP64 outputs in the face layout.  d_kx32, d_ky32: NULL,
 * or FP32 copies (needed by MSG_MIXED solves).  Errors: MSG_ERR_ARG (bad
 * spec, missing outputs, unknown face rule).  Enqueued on `stream`; returns
 * after it completes. */
msg_status msg_sample_field(msg_handle h, const msg_field_spec *spec, const msg_batch_desc *batch,
                            const double *d_xi, double *d_kx, double *d_ky,
                            float *d_kx32, float *d_ky32, msg_stream stream);

/* msg_sample_field for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops that forbid allocation).  Same
 * arguments and results as msg_sample_field; its device staging (per
 * sample about 32 bytes of tables plus 4 bytes per grid, and without d_xi
 * the drawn normals, 8 bytes per term) lives in a static array of 32 MiB
 * per device instead of memory allocated for the call; the call allocates
 * nothing.  Errors: those of msg_sample_field, and MSG_ERR_WORKSPACE, before
 * any device work, when a batch needs more than 32 MiB of staging (pass d_xi
 * or split the batch).  All calls on one device share that device's array
 * and nothing of a call survives in it that a later call needs: calls that
 * overlap on one device (other host threads, or another stream still
 * running one) race on it.  Returns after the work has completed on
 * `stream`. */
msg_status msg_sample_field_noalloc(msg_handle h, const msg_field_spec *spec, const msg_batch_desc *batch,
                                    const double *d_xi, double *d_kx, double *d_ky,
                                    float *d_kx32, float *d_ky32, msg_stream stream);

/* Full MSG solve of every sample (Section 2, Algorithm MSG F-cycle with the
 * MSG mu-cycle, eq. restriction, eq. interpolation, eq. weight_factors),
 * returning the solution of every grid (p,q) of every sample -- the coarse
 * solutions that Section 3 reuses at no extra cost in the multi-index
 * differences -- and Q = mean of u per grid.
 *   d_kx, d_ky      device FP64 face coefficients (msg_sample_field layout)
 *   d_kx32, d_ky32  device FP32 copies, required for MSG_MIXED, else ignored
 *   d_rhs           NULL for h = 1, else device FP64 right-hand side at the
 *                   cell centres of each sample's finest grid, packed per
 *                   sample (finest-grid cells only)
 *   d_u_out         device FP64 [cells] every grid's solution
 *   d_q_out         device FP64 [grids] mean of u over each grid
 *   d_status        device int32 [S] MSG_SAMPLE_*
 *   d_cycles        device int32 [grids] cycles run per grid (NULL allowed)
 *   d_ws, ws_bytes  device workspace of at least msg_workspace_size() bytes
 * Each grid (p,q), level by level from (0,0) up, starts from the weighted
 * cubic interpolation of the level below and runs mu-cycles over its own
 * rectangle [0..p]x[0..q] until ||r||_2 <= tol ||b||_2 or max_cycles.  A
 * sample whose norms turn non-finite gets status NONFINITE and NaN on the
 * grids of that level and above; other samples are unaffected.  The call
 * returns after the solve has completed on `stream` (it reads convergence
 * flags back between cycles). */
msg_status msg_solve_batch(msg_handle h, const msg_batch_desc *batch, const msg_solve_opts *opts,
                           const double *d_kx, const double *d_ky,
                           const float *d_kx32, const float *d_ky32,
                           const double *d_rhs, double *d_u_out, double *d_q_out,
                           int32_t *d_status, int32_t *d_cycles,
                           void *d_ws, size_t ws_bytes, msg_stream stream);

/* Quantities of interest per grid (Section 5 defines three for the unit
 * square; the readings below adapt them to the cell-centred grid):
 *   MSG_QOI_MEAN       mean of u over the cells (what msg_solve_batch returns in d_q_out);
 *   MSG_QOI_POINT      u(1/2,1/2): bilinear interpolation of the cell-centre values;
 *   MSG_QOI_SUBDOMAIN  average over D_sub = [1/4,1/2]^2 of the cell-wise constant solution,
 *                      each cell weighted by its area inside D_sub;
 *   MSG_QOI_FLUX       flux -int_0^1 k du/dx dy through the wall x = 1: per row, the wall
 *                      face's 2 k u / h_x (the one-sided difference of the discretisation)
 *                      times h_y.
 * d_u: device FP64 cells (msg_solve_batch layout); d_kx: device FP64 x-faces, required for
 * MSG_QOI_FLUX (else may be NULL); d_q: device FP64 [grids] output.  Enqueued on `stream`;
 * returns after it completes. */
enum { MSG_QOI_MEAN = 0, MSG_QOI_POINT = 1, MSG_QOI_SUBDOMAIN = 2, MSG_QOI_FLUX = 3 };
msg_status msg_quantity(const msg_batch_desc *batch, int kind, const double *d_kx, const double *d_u,
                        double *d_q, msg_stream stream);

/* Multi-index differences (Section 3): for every sample and grid l = (p,q),
 * Delta Q_l = (Delta_1 x Delta_2) Q_l with Delta_i Q_l = Q_l - Q_{l - e_i}
 * when l_i > 0, else Q_l.  d_q, d_dq: device FP64 [grids] in the per-grid
 * layout.  Enqueued on `stream`. */
msg_status mimc_delta_q(const msg_batch_desc *batch, const double *d_q, double *d_dq,
                        msg_stream stream);

/* Matern lognormal fields by circulant embedding (Section 1, eq. matern;
 * Section 5): k = exp(Z) with Z Gaussian, zero mean, covariance
 * C(r) = 2^(1-nu)/Gamma(nu) (2 sqrt(nu) r)^nu K_nu(2 sqrt(nu) r), r = |T (x1 - x2)|,
 * T = S R, S = diag(1/sqrt(eta lambda), 1/sqrt(lambda)), R the rotation by theta.
 * Each sample is drawn exactly on the lattice of half its finest mesh width
 * (which holds every face midpoint of every grid (p,q) <= (P,Q), so all grids
 * of a sample see one realisation) from a periodic embedding enlarged by
 * m = 1 + 2 ceil(sqrt(nu) log2(max(c 2^P, c 2^Q))) per direction (or `pad`),
 * rounded up to a power of two of at most 32768 points per direction (rows
 * above 8192 points, beyond one workgroup's LDS, run as the four-step FFT).  The
 * normals come from Philox4x64-10 with counter (frequency pair, sample id,
 * 0, 0) and key (seed, 0x6D617465726E), through u = ((w >> 12) + 1/2) 2^-52
 * and the Box-Muller transform.
 *   eta, theta: host [n_samples] (theta in radians; eta > 0), the paper's
 *               hyperparameters drawn per sample;
 *   sample_id:  host [n_samples] or NULL (0..n_samples-1): the random stream;
 * d_kx, d_ky (and optional FP32 copies): as msg_sample_field.  d_ratio: NULL
 * or device FP64 [n_samples], min/max eigenvalue of each sample's embedding;
 * a negative value means the embedding is indefinite (negative eigenvalues
 * are clamped to zero and that sample is approximate; raise `pad`).
 * Workspace: msg_matern_workspace_size bytes hold chunks of up to 8 samples;
 * any size that holds one sample of the largest embedding works, in more
 * chunks.  Errors: MSG_ERR_ARG, MSG_ERR_LAYOUT, MSG_ERR_UNSUPPORTED (an
 * embedding above 32768 points per direction), MSG_ERR_WORKSPACE.  Enqueued
 * on `stream`. */
typedef struct {
    double lambda;             /* length scale, > 0 */
    double nu;                 /* smoothness, 0 < nu <= 8 */
    const double *eta;         /* host [n_samples] */
    const double *theta;       /* host [n_samples] */
    const int64_t *sample_id;  /* host [n_samples] or NULL */
    uint64_t seed;
    int32_t pad;               /* 0: the paper's factor, else 1..64 */
    int32_t reserved;
} msg_matern_spec;
msg_status msg_matern_workspace_size(const msg_batch_desc *batch, const msg_matern_spec *spec,
                                     size_t *bytes);
msg_status msg_sample_matern(msg_handle h, const msg_matern_spec *spec, const msg_batch_desc *batch,
                             double *d_kx, double *d_ky, float *d_kx32, float *d_ky32,
                             double *d_ratio, void *d_ws, size_t ws_bytes, msg_stream stream);

/* Plain cycles from zero, the convergence-factor comparison of Section 2.
 * Every sample runs `ncycles` cycles on its finest grid (P,Q), started from
 * v = 0 with right-hand side h = 1 (d_rhs NULL) or d_rhs, and reports the
 * residual ratio ||h - A v_k|| / ||h|| (Euclidean norms over the cells)
 * before each cycle k = 0..ncycles.
 *   MSG_CYCLES_MSG  the mu-cycle of Algorithm MSG on the semi-coarsened
 *                   family (grids of every level below (P,Q));
 *   MSG_CYCLES_MG   standard multigrid: grid (p,q) coarsens to (p-1,q-1),
 *                   restriction is the average of the four fine cells of a
 *                   coarse cell, prolongation the bilinear interpolation of
 *                   the cell-centred iterate (odd reflection at the walls),
 *                   the operator is rediscretised on each grid from that
 *                   grid's face conductances, the coarsest grid (0,0) is
 *                   solved exactly, the smoother is the same red-black
 *                   Gauss-Seidel; requires P == Q.
 * Both use mu, nu1, nu2 and omega of `opts` (tol, max_cycles and the
 * adaptive rule are not used; every cycle runs); precision must be
 * MSG_FP64.  The batch must be uniform (one (P,Q) for every sample).
 * d_kx, d_ky: device FP64 faces (msg_sample_field layout).  d_rhs: NULL or
 * device FP64 [n_samples][finest cells], sample-major.  d_u_top: device FP64
 * [n_samples][finest cells], the iterate after the last cycle.  d_ratios:
 * device FP64 [n_samples][ncycles + 1].  Workspace from
 * msg_cycles_workspace_size (whose handle may be NULL; 256-byte aligned).  Errors: MSG_ERR_ARG (bad
 * pointer, kind, ncycles outside 0..10000), MSG_ERR_UNSUPPORTED (ragged
 * batch, P != Q for MG, precision other than FP64, a tail that does not fit
 * LDS), MSG_ERR_WORKSPACE.  Enqueued on `stream`; returns after it completes. */
enum { MSG_CYCLES_MSG = 0, MSG_CYCLES_MG = 1 };
msg_status msg_cycles_workspace_size(msg_handle h, const msg_batch_desc *batch, const msg_solve_opts *opts,
                                     int kind, size_t *bytes);
msg_status msg_cycles(msg_handle h, const msg_batch_desc *batch, const msg_solve_opts *opts, int kind,
                      int ncycles, const double *d_kx, const double *d_ky, const double *d_rhs,
                      double *d_u_top, double *d_ratios, void *d_ws, size_t ws_bytes, msg_stream stream);

/* Per-kernel timing (measurement support).  While enabled, msg_solve_batch
 * records a pair of HIP events around every launch of each kernel kind on
 * the stream it runs on and accumulates, per kind, the launches, the summed
 * event time and the algorithmic bytes of those launches (the data the
 * kernel must touch at least once for the problems still cycling).  With
 * overlap, launches of different classes may share the device, and their
 * event times include that sharing.  The two *_STAGE kinds are subsets of
 * SMOOTH and RESTRICT: the launches on the F-cycle stage's own level, whose
 * grids are the largest of the stage and stream from HBM.  Enabling or
 * disabling clears the totals. */
enum {
    MSG_KERNEL_SMOOTH = 0,        /* red-black Gauss-Seidel passes (with nu1 = 2 the
                                     pre-smoothing pass also restricts its residual) */
    MSG_KERNEL_RESTRICT = 1,      /* residual + restriction (eq. restriction); where the
                                     pre-smoothing pass restricts its own residual (nu1 = 2),
                                     only the combination on coarse grids with two parents */
    MSG_KERNEL_PROLONG = 2,       /* weighted correction (eq. interpolation) */
    MSG_KERNEL_TAIL = 3,          /* on-chip cycles of the lowest levels */
    MSG_KERNEL_RESIDUAL_NORM = 4, /* finest-grid residual norms */
    MSG_KERNEL_SMOOTH_STAGE = 5,  /* SMOOTH launches on the stage's own level */
    MSG_KERNEL_RESTRICT_STAGE = 6,/* RESTRICT launches from the stage's own level */
    MSG_KERNEL_KINDS = 7
};
typedef struct {
    int64_t launches;
    double milliseconds;          /* sum of per-launch event times */
    double bytes;                 /* algorithmic bytes of those launches */
    double model_bytes;           /* the per-step byte model: every red-black sweep reads v, b
                                     and the conductances and writes v as a step of its own
                                     (5 values per cell), and so do the residual with its
                                     restriction and the coarse-grid correction; equal to
                                     `bytes` for kinds other than MSG_KERNEL_SMOOTH */
} msg_kernel_stats;

/* enable: 0 off, 1 an event pair around every launch, n > 1 around one
 * launch in n (picked by a hash of a running launch counter, so the choice
 * does not follow the regular launch pattern of a cycle).  Sampled totals
 * are scaled to every launch: `launches` counts all launches of the kind,
 * `milliseconds` and `bytes` are the timed launches' sums times (all /
 * timed), so averages and bytes per millisecond are those of the timed
 * launches (both zero for a kind none of whose launches was timed).
 * MSG_ERR_ARG for a negative rate. */
msg_status msg_set_profiling(msg_handle h, int enable);
msg_status msg_get_profile(msg_handle h, int kind, msg_kernel_stats *out);

#ifdef __cplusplus
}
#endif
#endif
