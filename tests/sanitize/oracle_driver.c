/* Runs every entry point of the C oracle on small seeded problems, built
 * together with oracle/msg_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py).  Any out-of-bounds
 * access, use after free, leak or undefined operation aborts the run; the
 * driver itself checks only that the solves converge and the outputs are
 * finite.  Prints "oracle driver ok" at the end. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t mu, nu1, nu2, max_cycles;
    double tol, omega;
    int32_t joint_stages;
} oracle_opts;

int oracle_fmsg_solve(int c, int P, int Q, const double *kx_all, const double *ky_all, const double *rhs_top,
                      const oracle_opts *o, const int32_t *forced_cycles, double *u_out, double *q_out,
                      int32_t *cycles_out, double *hist);
void oracle_msg_cycles(int c, int P, int Q, const double *kx_all, const double *ky_all, const double *rhs_top,
                       const oracle_opts *o, int ncycles, double *u_top, double *ratios);
void oracle_mg_cycles(int c, int P, int Q, const double *kx_all, const double *ky_all, const double *rhs_top,
                      const oracle_opts *o, int ncycles, double *u_top, double *ratios);
void oracle_delta_q(int P, int Q, const double *q, double *dq);
double oracle_qoi_grid(int nx, int ny, const double *kx, const double *u, int kind);
void oracle_apply(int nx, int ny, const double *kx, const double *ky, const double *u, double *out);
void oracle_residual(int nx, int ny, const double *kx, const double *ky, const double *b, const double *u,
                     double *r);
void oracle_rbgs(int nx, int ny, const double *kx, const double *ky, const double *b, double *u, int sweeps);
void oracle_weights(int nx, int ny, const double *kx, const double *ky, double *kap_x, double *kap_y);
void oracle_restrict_x(int nxc, int ny, const double *fine, double *coarse);
void oracle_restrict_y(int nx, int nyc, const double *fine, double *coarse);
void oracle_prolong_x(int nxc, int ny, const double *coarse, double *fine, int cubic);
void oracle_prolong_y(int nx, int nyc, const double *coarse, double *fine, int cubic);
void oracle_correction(int c, int p, int q, const double *kx, const double *ky, const double *e_x,
                       const double *e_y, int cubic, double *out);
void oracle_field_cos(int nx, int ny, int nterms, const int32_t *a, const int32_t *b, const double *amp,
                      const double *xi, double *kx, double *ky);
void oracle_face_mean(int c, int P, int Q, const double *kxF, const double *kyF, int p, int q, double *kx,
                      double *ky);
void oracle_field_separable(int nx, int ny, int mx, int my, double lenx, double leny, double sigma2,
                            const double *xi, double *kx, double *ky);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double uniform(void)           /* xorshift64*, in [0, 1) */
{
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (double)((rng_state * 2685821657736338717ull) >> 11) * 0x1.0p-53;
}
static double normal(void) { return sqrt(-2.0 * log(1.0 - uniform())) * cos(6.283185307179586 * uniform()); }

static void *xmalloc(size_t n)
{
    void *p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static int failures = 0;
static void check(int ok, const char *what, int c, int P, int Q)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s at c=%d P=%d Q=%d\n", what, c, P, Q);
        ++failures;
    }
}
static int all_finite(const double *x, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

static void run_case(int c, int P, int Q)
{
    static const int32_t ta[10] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0};
    static const int32_t tb[10] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3};
    double amp[10], xi[10];
    for (int t = 0; t < 10; ++t) {
        amp[t] = 1.0 / (t + 1);
        xi[t] = normal();
    }
    const int G = (P + 1) * (Q + 1);
    size_t ncell = 0, nxf = 0, nyf = 0;
    for (int p = 0; p <= P; ++p)
        for (int q = 0; q <= Q; ++q) {
            const size_t nx = (size_t)c << p, ny = (size_t)c << q;
            ncell += nx * ny;
            nxf += (nx + 1) * ny;
            nyf += nx * (ny + 1);
        }
    double *kx = xmalloc(nxf * sizeof(double)), *ky = xmalloc(nyf * sizeof(double));
    size_t ox = 0, oy = 0;
    for (int p = 0; p <= P; ++p)
        for (int q = 0; q <= Q; ++q) {
            const int nx = c << p, ny = c << q;
            oracle_field_cos(nx, ny, 10, ta, tb, amp, xi, kx + ox, ky + oy);
            ox += (size_t)(nx + 1) * ny;
            oy += (size_t)nx * (ny + 1);
        }
    check(all_finite(kx, nxf) && all_finite(ky, nyf), "field", c, P, Q);

    const oracle_opts o = {2, 2, 2, 60, 1e-10, 1.0, 0};
    double *u = xmalloc(ncell * sizeof(double));
    double *qv = xmalloc(G * sizeof(double)), *dq = xmalloc(G * sizeof(double));
    int32_t *cyc = xmalloc(G * sizeof(int32_t));
    double *hist = xmalloc((size_t)G * (o.max_cycles + 1) * sizeof(double));
    const int st = oracle_fmsg_solve(c, P, Q, kx, ky, NULL, &o, NULL, u, qv, cyc, hist);
    check(st == 0 && all_finite(u, ncell) && all_finite(qv, G), "fmsg solve", c, P, Q);
    oracle_delta_q(P, Q, qv, dq);
    check(all_finite(dq, G), "delta q", c, P, Q);

    /* forced cycle counts, a test right-hand side, the joint-level reading */
    int32_t *forced = xmalloc(G * sizeof(int32_t));
    for (int g = 0; g < G; ++g) forced[g] = 1 + g % 3;
    const size_t ntop = ((size_t)c << P) * ((size_t)c << Q);
    double *rhs = xmalloc(ntop * sizeof(double));
    for (size_t i = 0; i < ntop; ++i) rhs[i] = normal();
    oracle_fmsg_solve(c, P, Q, kx, ky, rhs, &o, forced, u, qv, cyc, NULL);
    check(all_finite(u, ncell), "forced cycles", c, P, Q);
    const oracle_opts oj = {1, 1, 1, 3, 1e-10, 0.8, 1};
    oracle_fmsg_solve(c, P, Q, kx, ky, NULL, &oj, NULL, u, qv, cyc, NULL);
    check(all_finite(u, ncell), "joint stages", c, P, Q);

    /* plain cycles from zero on the finest grid */
    double *utop = xmalloc(ntop * sizeof(double)), *ratios = xmalloc(6 * sizeof(double));
    oracle_msg_cycles(c, P, Q, kx, ky, NULL, &o, 5, utop, ratios);
    check(all_finite(ratios, 6) && ratios[5] < ratios[0], "msg cycles", c, P, Q);
    if (P == Q) {
        oracle_mg_cycles(c, P, Q, kx, ky, rhs, &o, 5, utop, ratios);
        check(all_finite(ratios, 6), "mg cycles", c, P, Q);
    }

    /* the finest grid's pieces, face means and the correction of every grid */
    const int nx = c << P, ny = c << Q;
    const double *kxF = kx + ox - (size_t)(nx + 1) * ny, *kyF = ky + oy - (size_t)nx * (ny + 1);
    const double *uF = u + ncell - ntop;
    for (int kind = 0; kind < 4; ++kind) check(isfinite(oracle_qoi_grid(nx, ny, kxF, uF, kind)), "qoi", c, P, Q);
    const size_t nface = (size_t)(nx + 1) * (ny + 1);      /* holds the cells or either face set of a grid */
    double *w1 = xmalloc(nface * sizeof(double)), *w2 = xmalloc(nface * sizeof(double));
    oracle_apply(nx, ny, kxF, kyF, uF, w1);
    oracle_residual(nx, ny, kxF, kyF, rhs, uF, w2);
    memcpy(w1, uF, ntop * sizeof(double));
    oracle_rbgs(nx, ny, kxF, kyF, rhs, w1, 2);
    oracle_weights(nx, ny, kxF, kyF, w1, w2);
    check(all_finite(w1, ntop) && all_finite(w2, ntop), "grid operators", c, P, Q);
    double *cx = xmalloc(ntop * sizeof(double)), *cy = xmalloc(ntop * sizeof(double));
    if (P > 0) {
        oracle_restrict_x(nx / 2, ny, uF, cx);
        for (int cubic = 0; cubic < 2; ++cubic) oracle_prolong_x(nx / 2, ny, cx, w1, cubic);
    }
    if (Q > 0) {
        oracle_restrict_y(nx, ny / 2, uF, cy);
        for (int cubic = 0; cubic < 2; ++cubic) oracle_prolong_y(nx, ny / 2, cy, w2, cubic);
    }
    if (P > 0 || Q > 0)
        for (int cubic = 0; cubic < 2; ++cubic) {
            oracle_correction(c, P, Q, kxF, kyF, P > 0 ? cx : NULL, Q > 0 ? cy : NULL, cubic, w1);
            check(all_finite(w1, ntop), "correction", c, P, Q);
        }
    for (int p = 0; p <= P; ++p)
        for (int q = 0; q <= Q; ++q) {
            const size_t gx = (size_t)c << p, gy = (size_t)c << q;
            oracle_face_mean(c, P, Q, kxF, kyF, p, q, w1, w2);
            check(all_finite(w1, (gx + 1) * gy) && all_finite(w2, gx * (gy + 1)), "face mean", c, P, Q);
        }
    double sxi[36];
    for (int t = 0; t < 36; ++t) sxi[t] = normal();
    oracle_field_separable(nx, ny, 6, 6, 0.3, 0.05, 1.0, sxi, w1, w2);
    check(all_finite(w1, (size_t)(nx + 1) * ny) && all_finite(w2, (size_t)nx * (ny + 1)), "separable", c, P, Q);

    free(kx); free(ky); free(u); free(qv); free(dq); free(cyc); free(hist); free(forced); free(rhs);
    free(utop); free(ratios); free(w1); free(w2); free(cx); free(cy);
}

int main(void)
{
    static const int cases[][3] = {{1, 0, 0}, {2, 0, 3}, {2, 3, 0}, {2, 3, 3}, {4, 2, 3}, {4, 1, 1},
                                   {3, 2, 2}, {8, 1, 0}, {4, 4, 2}};
    for (size_t k = 0; k < sizeof cases / sizeof cases[0]; ++k) run_case(cases[k][0], cases[k][1], cases[k][2]);
    if (failures) return 1;
    printf("oracle driver ok\n");
    return 0;
}
