// matern.hip -- Matern Gaussian random fields by circulant embedding on
// gfx950: the coefficient k = exp(Z) of Section 1 with the covariance of
// eq. matern (distance r = |T (x1 - x2)|, T = S R with S = diag(1/sqrt(eta
// lambda), 1/sqrt(lambda)) and R the rotation by theta), sampled exactly as in
// Section 5 on a periodic domain enlarged by 1 + 2 ceil(sqrt(nu) log2 n).
//
// One sample of Z on the lattice of half the finest mesh width holds every
// face midpoint of every grid of the sample.  Per sample (several at once,
// one launch per step for all of them):
//   1. the first row of the block-circulant embedding, c[iy][ix], from the
//      covariance at the wrapped displacements (both signs averaged on the
//      half-period lines, which keeps the matrix symmetric);
//   2. its 2D DFT (the eigenvalues Lambda): radix-2 FFTs of whole rows in LDS,
//      one workgroup per row, a tiled transpose, FFTs of the other direction;
//      Lambda stays transposed;
//   3. min and max of Lambda (the positive-definiteness check);
//   4. W = sqrt(max(Lambda, 0) / M) xi with complex standard normal xi from
//      Philox4x64-10 (Salmon et al., SC 2011) and the Box-Muller transform,
//      indexed by the frequency's row-major position;
//   5. the 2D DFT of W back in row-major order (FFTs, transpose, FFTs);
//   6. k = exp(Re Y) at every x- and y-face midpoint of every grid, in the
//      library's face layout (and FP32 copies when asked for).
// The DFT is the forward one, exp(-2 pi i jk / N), unnormalised.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

#include "matern_kernels.hpp"
#include "msg_device.hpp"
#include "philox.hpp"

namespace msg {

#define LAUNCH_CHECK() hipGetLastError()

// ------------------------------------------------------------------ covariance
// K_nu(z) by the trapezoidal rule on K_nu(z) = int_0^inf exp(-z cosh t)
// cosh(nu t) dt (the integrand is entire and decays doubly exponentially, so
// the rule converges geometrically in the step); summed until the terms fall
// 40 e-folds below the largest one.
__device__ double bessel_k(double nu, double z)
{
    const double h = 0.125;
    const double tpk = asinh(nu / z);                        // where the log-integrand peaks
    const double peak = -z * cosh(tpk) + nu * tpk;
    double sum = 0.5 * exp(-z);                              // t = 0 (cosh 0 = 1), half weight
    for (int k = 1; k < 4096; ++k) {
        const double t = k * h;
        const double e = -z * cosh(t);
        const double lg = e + nu * t;
        sum += 0.5 * (exp(lg) + exp(e - nu * t));
        if (t > tpk && lg < peak - 40.0) break;
    }
    return h * sum;
}

__device__ double matern_cov(const MaternSample& S, double nu, double coef, double dx, double dy)
{
    const double tx = S.t00 * dx + S.t01 * dy;
    const double ty = S.t10 * dx + S.t11 * dy;
    const double r = sqrt(tx * tx + ty * ty);
    if (r == 0.0) return 1.0;
    const double z = 2.0 * sqrt(nu) * r;
    if (nu == 0.5) return exp(-z);                           // 2^(1/2)/Gamma(1/2) z^(1/2) K_(1/2)(z) = e^-z
    if (z > 745.0) return 0.0;
    return coef * pow(z, nu) * bessel_k(nu, z);
}

__global__ void __launch_bounds__(256)
k_mat_row(int Mx, int My, double hx, double hy, double nu, double coef, const MaternSample* __restrict__ smp,
          double2* __restrict__ A)
{
    const int s = blockIdx.y;
    const int64_t M = (int64_t)Mx * My;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M) return;
    const MaternSample S = smp[s];
    const int ix = (int)(idx % Mx), iy = (int)(idx / Mx);
    const int dx = ix <= Mx / 2 ? ix : ix - Mx;
    const int dy = iy <= My / 2 ? iy : iy - My;
    const bool hx_line = ix == Mx / 2, hy_line = iy == My / 2;
    double c = matern_cov(S, nu, coef, dx * hx, dy * hy);
    if (hx_line && hy_line) {
        c = 0.25 * (2.0 * c + 2.0 * matern_cov(S, nu, coef, -dx * hx, dy * hy));
    } else if (hx_line) {
        c = 0.5 * (c + matern_cov(S, nu, coef, -dx * hx, dy * hy));
    } else if (hy_line) {
        c = 0.5 * (c + matern_cov(S, nu, coef, dx * hx, -dy * hy));
    }
    A[(int64_t)s * M + idx] = make_double2(c, 0.0);
}

// ------------------------------------------------------------------ FFT
__global__ void __launch_bounds__(256)
k_twiddles(int n_max, double2* __restrict__ tw)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_max / 2) return;
    double s, c;
    sincospi(-2.0 * (double)k / (double)n_max, &s, &c);
    tw[k] = make_double2(c, s);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place radix-2 FFT of rows of length N = 2^logn (one workgroup per row):
// bit-reversed load into LDS, log2 N butterfly stages, store.  tw holds
// exp(-2 pi i k / n_max) for k < n_max / 2; this length uses every
// (n_max / N)-th entry.
__global__ void __launch_bounds__(256)
k_fft_rows(int64_t rows, int logn, int tw_stride, const double2* __restrict__ tw, double2* __restrict__ X)
{
    extern __shared__ double2 buf[];
    const int64_t row = blockIdx.x;
    if (row >= rows) return;
    const int N = 1 << logn;
    double2* x = X + row * N;
    for (int i = threadIdx.x; i < N; i += blockDim.x) buf[__brev((unsigned)i) >> (32 - logn)] = x[i];
    __syncthreads();
    for (int lg = 1; lg <= logn; ++lg) {
        const int half = 1 << (lg - 1);
        const int step = (N >> lg) * tw_stride;
        for (int b = threadIdx.x; b < N / 2; b += blockDim.x) {
            const int pos = b & (half - 1);
            const int i = ((b >> (lg - 1)) << lg) + pos;
            const double2 u = buf[i];
            const double2 v = cmul(buf[i + half], tw[pos * step]);
            buf[i] = make_double2(u.x + v.x, u.y + v.y);
            buf[i + half] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < N; i += blockDim.x) x[i] = buf[i];
}

// Rows longer than one workgroup's LDS holds (four-step FFT, Bailey 1990):
// a row of N = N1 N2 points, x[N2 n1 + n2], is an N1 x N2 matrix; after the
// transpose to [n2][n1] and length-N1 FFTs of its rows, entry [n2][k1] is
// multiplied by exp(-2 pi i n2 k1 / N); after the transpose to [k1][n2] and
// length-N2 FFTs, entry [k1][k2] holds X[k1 + N1 k2], and a last transpose
// puts it in natural order.  This kernel is the twiddle step, over
// rows x N2 x N1 entries.
__global__ void __launch_bounds__(256)
k_fft_twiddle(int64_t total, int logn, int h1, double2* __restrict__ X)
{
    const int64_t N = (int64_t)1 << logn;
    const int64_t n1mask = ((int64_t)1 << h1) - 1;
    const int64_t n2mask = (N >> h1) - 1;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k1 = e & n1mask, n2 = (e >> h1) & n2mask;
        const int64_t m = (n2 * k1) & (N - 1);
        double s, c;
        sincospi(-2.0 * (double)m / (double)N, &s, &c);
        X[e] = cmul(X[e], make_double2(c, s));
    }
}

// out[s][c][r] = in[s][r][c] for R x C complex matrices, 32 x 32 tiles
__global__ void __launch_bounds__(256)
k_transpose(int R, int C, const double2* __restrict__ in, double2* __restrict__ out)
{
    __shared__ double2 tile[32][33];
    const int64_t off = (int64_t)blockIdx.z * R * C;
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int r = r0 + k, c = c0 + threadIdx.x;
        if (r < R && c < C) tile[k][threadIdx.x] = in[off + (int64_t)r * C + c];
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int c = c0 + k, r = r0 + threadIdx.x;
        if (r < R && c < C) out[off + (int64_t)c * R + r] = tile[threadIdx.x][k];
    }
}

// ------------------------------------------------------------------ eigenvalues
__global__ void __launch_bounds__(256)
k_eig_minmax(int64_t M, int nb, const double2* __restrict__ L, double2* __restrict__ part)
{
    __shared__ double lo[256], hi[256];
    const int s = blockIdx.y;
    const double2* l = L + (int64_t)s * M;
    double a = INFINITY, b = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)nb * blockDim.x) {
        const double v = l[i].x;
        a = fmin(a, v);
        b = fmax(b, v);
    }
    lo[threadIdx.x] = a;
    hi[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            lo[threadIdx.x] = fmin(lo[threadIdx.x], lo[threadIdx.x + w]);
            hi[threadIdx.x] = fmax(hi[threadIdx.x], hi[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)s * nb + blockIdx.x] = make_double2(lo[0], hi[0]);
}

__global__ void __launch_bounds__(64)
k_eig_ratio(int nb, const double2* __restrict__ part, const int32_t* __restrict__ out_index,
            double* __restrict__ ratio)
{
    const int s = blockIdx.x;
    double a = INFINITY, b = -INFINITY;
    for (int i = threadIdx.x; i < nb; i += 64) {
        const double2 v = part[(int64_t)s * nb + i];
        a = fmin(a, v.x);
        b = fmax(b, v.y);
    }
    for (int off = 32; off > 0; off >>= 1) {
        a = fmin(a, __shfl_down(a, off, 64));
        b = fmax(b, __shfl_down(b, off, 64));
    }
    if (threadIdx.x == 0) ratio[out_index[s]] = a / b;
}

// ------------------------------------------------------------------ normals
// Philox4x64-10 and uniform52: philox.hpp

// W = sqrt(max(Lambda, 0) / M) xi on the transposed layout [kx][ky]; xi of
// the frequency at row-major position l = ky Mx + kx is the Box-Muller pair
// of words (0,1) (l even) or (2,3) (l odd) of Philox at counter (l / 2, id).
__global__ void __launch_bounds__(256)
k_mat_xi(int Mx, int My, uint64_t seed, uint64_t key1, const MaternSample* __restrict__ smp,
         double2* __restrict__ LT)
{
    const int s = blockIdx.y;
    const int64_t M = (int64_t)Mx * My;
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= M) return;
    const int kx = (int)(pos / My), ky = (int)(pos % My);
    const int64_t l = (int64_t)ky * Mx + kx;
    uint64_t c[4] = {(uint64_t)(l >> 1), (uint64_t)smp[s].id, 0, 0};
    philox4x64_10(c, seed, key1);
    const uint64_t wa = (l & 1) ? c[2] : c[0], wb = (l & 1) ? c[3] : c[1];
    const double rho = sqrt(-2.0 * log(uniform52(wa)));
    double sn, cs;
    sincos(2.0 * M_PI * uniform52(wb), &sn, &cs);
    double2* e = LT + (int64_t)s * M + pos;
    const double lam = (*e).x;
    const double a = sqrt(fmax(lam, 0.0) / (double)M);
    *e = make_double2(a * rho * cs, a * rho * sn);
}

// ------------------------------------------------------------------ faces
// k = exp(Re Y) at the faces of grid (p,q) = (g / (Q+1), g % (Q+1)) of every
// sample of the chunk (all of rectangle (P,Q)); Y is row-major [b][a] on the
// embedding lattice, face (i/nx, (j+1/2)/ny) at a = i 2^(P-p+1), b = (2j+1)
// 2^(Q-q), face ((i+1/2)/nx, j/ny) at a = (2i+1) 2^(P-p), b = j 2^(Q-q+1).
__global__ void __launch_bounds__(256)
k_mat_faces(int c, int P, int Q, int Mx, int My, const MaternSample* __restrict__ smp, const double2* __restrict__ Y,
            double* __restrict__ kx, double* __restrict__ ky, float* __restrict__ kx32, float* __restrict__ ky32)
{
    const int g = blockIdx.y, s = blockIdx.z;
    const int p = g / (Q + 1), q = g % (Q + 1);
    const int nx = c << p, ny = c << q;
    const int64_t nfx = (int64_t)(nx + 1) * ny, nfy = (int64_t)nx * (ny + 1);
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double2* y = Y + (int64_t)s * Mx * My;
    const MaternSample S = smp[s];
    if (idx < nfx) {
        const int i = (int)(idx % (nx + 1)), j = (int)(idx / (nx + 1));
        const int64_t a = (int64_t)i << (P - p + 1), b = (int64_t)(2 * j + 1) << (Q - q);
        const double v = exp(y[b * Mx + a].x);
        const int64_t o = S.fx_base + xface_off(c, Q, p, q) + idx;
        kx[o] = v;
        if (kx32) kx32[o] = (float)v;
    }
    if (idx < nfy) {
        const int i = (int)(idx % nx), j = (int)(idx / nx);
        const int64_t a = (int64_t)(2 * i + 1) << (P - p), b = (int64_t)j << (Q - q + 1);
        const double v = exp(y[b * Mx + a].x);
        const int64_t o = S.fy_base + yface_off(c, Q, p, q) + idx;
        ky[o] = v;
        if (ky32) ky32[o] = (float)v;
    }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_mat_twiddles(int n_max, double2* tw, hipStream_t st)
{
    hipLaunchKernelGGL(k_twiddles, dim3((n_max / 2 + 255) / 256), dim3(256), 0, st, n_max, tw);
    return LAUNCH_CHECK();
}

hipError_t launch_mat_row(int K, int Mx, int My, double hx, double hy, double nu, double coef,
                          const MaternSample* smp, double2* A, hipStream_t st)
{
    const int64_t M = (int64_t)Mx * My;
    hipLaunchKernelGGL(k_mat_row, dim3((unsigned)((M + 255) / 256), K), dim3(256), 0, st, Mx, My, hx, hy, nu, coef,
                       smp, A);
    return LAUNCH_CHECK();
}

hipError_t launch_fft_rows(int64_t rows, int logn, int tw_stride, const double2* tw, double2* X, hipStream_t st)
{
    const size_t lds = sizeof(double2) << logn;
    if (lds > 65536) {                        // rows of 8192 points: 128 KB of the CU's 160 KB
        hipError_t e = hipFuncSetAttribute((const void*)k_fft_rows, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_fft_rows, dim3((unsigned)rows), dim3(256), lds, st, rows, logn, tw_stride, tw, X);
    return LAUNCH_CHECK();
}

hipError_t launch_transpose(int K, int R, int C, const double2* in, double2* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_transpose, dim3((C + 31) / 32, (R + 31) / 32, K), dim3(32, 8), 0, st, R, C, in, out);
    return LAUNCH_CHECK();
}

// K matrices of R x C, in slices of at most 32768 (the grid's z limit)
static hipError_t transpose_many(int64_t K, int R, int C, const double2* in, double2* out, hipStream_t st)
{
    const int64_t per = (int64_t)R * C;
    for (int64_t k0 = 0; k0 < K; k0 += 32768) {
        const int kn = (int)std::min<int64_t>(32768, K - k0);
        hipError_t e = launch_transpose(kn, R, C, in + k0 * per, out + k0 * per, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fft_rows_long(int64_t rows, int logn, int h1, int tw_log, const double2* tw, double2* X,
                                double2* S, hipStream_t st)
{
    const int h2 = logn - h1;
    const int N1 = 1 << h1, N2 = 1 << h2;
    const int64_t total = rows << logn;
    hipError_t e;
    if ((e = transpose_many(rows, N1, N2, X, S, st)) != hipSuccess) return e;               // [n2][n1]
    if ((e = launch_fft_rows(rows * N2, h1, (1 << tw_log) >> h1, tw, S, st)) != hipSuccess) return e;
    const int64_t blocks = std::min<int64_t>((total + 255) / 256, (int64_t)1 << 20);
    hipLaunchKernelGGL(k_fft_twiddle, dim3((unsigned)blocks), dim3(256), 0, st, total, logn, h1, S);
    if ((e = LAUNCH_CHECK()) != hipSuccess) return e;
    if ((e = transpose_many(rows, N2, N1, S, X, st)) != hipSuccess) return e;               // [k1][n2]
    if ((e = launch_fft_rows(rows * N1, h2, (1 << tw_log) >> h2, tw, X, st)) != hipSuccess) return e;
    if ((e = transpose_many(rows, N1, N2, X, S, st)) != hipSuccess) return e;               // [k2][k1]
    return hipMemcpyAsync(X, S, sizeof(double2) * (size_t)total, hipMemcpyDeviceToDevice, st);
}

hipError_t launch_eig_ratio(int K, int64_t M, int nb, const double2* L, double2* part, const int32_t* out_index,
                            double* ratio, hipStream_t st)
{
    hipLaunchKernelGGL(k_eig_minmax, dim3(nb, K), dim3(256), 0, st, M, nb, L, part);
    hipError_t e = LAUNCH_CHECK();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_eig_ratio, dim3(K), dim3(64), 0, st, nb, part, out_index, ratio);
    return LAUNCH_CHECK();
}

hipError_t launch_mat_xi(int K, int Mx, int My, uint64_t seed, uint64_t key1, const MaternSample* smp, double2* LT,
                         hipStream_t st)
{
    const int64_t M = (int64_t)Mx * My;
    hipLaunchKernelGGL(k_mat_xi, dim3((unsigned)((M + 255) / 256), K), dim3(256), 0, st, Mx, My, seed, key1, smp, LT);
    return LAUNCH_CHECK();
}

hipError_t launch_mat_faces(int K, int c, int P, int Q, int Mx, int My, const MaternSample* smp, const double2* Y,
                            double* kx, double* ky, float* kx32, float* ky32, hipStream_t st)
{
    const int64_t nx = (int64_t)c << P, ny = (int64_t)c << Q;
    const int64_t most = (nx + 1) * (ny + 1);
    hipLaunchKernelGGL(k_mat_faces, dim3((unsigned)((most + 255) / 256), (P + 1) * (Q + 1), K), dim3(256), 0, st, c, P,
                       Q, Mx, My, smp, Y, kx, ky, kx32, ky32);
    return LAUNCH_CHECK();
}

}  // namespace msg
