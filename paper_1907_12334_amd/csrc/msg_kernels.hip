// msg_kernels.hip -- CDNA4 (gfx950) kernels of the batched MSG solver.
//
// Paper: Robbe, Nuyens, Vandewalle, arXiv 1907.12334, Section 2 (MSG), with
// the cell-centred finite-volume discretisation described in include/msg.h.
//
// Every stencil kernel here is memory-bound (a handful of flops per 8-byte
// value), so the design goals are coalesced row-major access, LDS tiles with
// recomputed halos for the smoother, and one block per tile of one grid of
// one problem so that a launch covers the whole batch.  No MFMA: there is no
// dense contraction on the path.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "msg_device.hpp"
#include "msg_kernels.hpp"
#include "philox.hpp"

namespace msg {

// ------------------------------------------------------------------------
// 5-point cell-centred finite-volume operator (Section 1, eq. PDE): the flux
// through a face is its conductance k/h^2 times the jump; a wall face is half
// a cell from the Dirichlet wall (u = 0), so its conductance doubles.
// ------------------------------------------------------------------------
template <typename T>
struct Stencil {
    T wW, wE, wS, wN;
};

template <typename T>
__device__ __forceinline__ Stencil<T> stencil_at(const T* __restrict__ kx, const T* __restrict__ ky, int nx, int ny,
                                                 int i, int j, T ihx2, T ihy2)
{
    Stencil<T> s;
    s.wW = kx[(int64_t)j * (nx + 1) + i] * ihx2;
    s.wE = kx[(int64_t)j * (nx + 1) + i + 1] * ihx2;
    s.wS = ky[(int64_t)j * nx + i] * ihy2;
    s.wN = ky[(int64_t)(j + 1) * nx + i] * ihy2;
    if (i == 0) s.wW *= T(2);
    if (i == nx - 1) s.wE *= T(2);
    if (j == 0) s.wS *= T(2);
    if (j == ny - 1) s.wN *= T(2);
    return s;
}

// r = b - A v at cell (i,j) of a grid stored row-major in global memory
template <typename T>
__device__ __forceinline__ T residual_at(const T* __restrict__ v, const T* __restrict__ b, const T* __restrict__ kx,
                                         const T* __restrict__ ky, int nx, int ny, int i, int j, T ihx2, T ihy2)
{
    const Stencil<T> s = stencil_at(kx, ky, nx, ny, i, j, ihx2, ihy2);
    const int64_t c = (int64_t)j * nx + i;
    const T u = v[c];
    const T uW = i > 0 ? v[c - 1] : T(0);
    const T uE = i < nx - 1 ? v[c + 1] : T(0);
    const T uS = j > 0 ? v[c - nx] : T(0);
    const T uN = j < ny - 1 ? v[c + nx] : T(0);
    return b[c] - (s.wW * (u - uW) + s.wE * (u - uE) + s.wS * (u - uS) + s.wN * (u - uN));
}

// One Gauss-Seidel update of a cell from its neighbours (zero beyond a wall):
// the fused smoother and the one-colour kernel share this arithmetic, so the
// two agree bit for bit.
template <typename T>
__device__ __forceinline__ T gs_update(const Stencil<T>& s, T b, T vW, T vE, T vS, T vN)
{
    const T num = b + s.wW * vW + s.wE * vE + s.wS * vS + s.wN * vN;
    return num / (s.wW + s.wE + s.wS + s.wN);
}

// Weight factors (eq. weight_factors) in closed form: with f = (-1)^i,
// (A f)_ij = (-1)^i [2 (kW + kE)/hx^2 + 2 k_wall/hy^2 on cells touching a
// y-wall]; symmetrically for g = (-1)^j.  kappa_x = lx^2 / (lx^2 + ly^2).
template <typename T>
__device__ __forceinline__ T kappa_x_at(const T* __restrict__ kx, const T* __restrict__ ky, int nx, int ny, int i,
                                        int j, T ihx2, T ihy2)
{
    const T kW = kx[(int64_t)j * (nx + 1) + i], kE = kx[(int64_t)j * (nx + 1) + i + 1];
    const T kS = ky[(int64_t)j * nx + i], kN = ky[(int64_t)(j + 1) * nx + i];
    T lx = T(2) * (kW + kE) * ihx2;
    T ly = T(2) * (kS + kN) * ihy2;
    if (j == 0) lx += T(2) * kS * ihy2;
    if (j == ny - 1) lx += T(2) * kN * ihy2;
    if (i == 0) ly += T(2) * kW * ihx2;
    if (i == nx - 1) ly += T(2) * kE * ihx2;
    const T a = lx * lx, c = ly * ly;
    return a / (a + c);
}

// value of a coarse line at index I with odd reflection at both walls
template <typename T>
__device__ __forceinline__ T odd_at(const T* __restrict__ line, int64_t stride, int n, int I)
{
    T sign = T(1);
    while (I < 0 || I >= n) {
        I = I < 0 ? -1 - I : 2 * n - 1 - I;
        sign = -sign;
    }
    return sign * line[(int64_t)I * stride];
}

// cell-centred linear interpolation (3/4, 1/4) of fine index i (0 <= i < 2n)
// from a coarse line of n values; the neighbour is at most one cell outside
// the line, where the odd reflection is minus the edge value itself
template <typename T>
__device__ __forceinline__ T linear_at(const T* __restrict__ line, int64_t stride, int n, int i)
{
    const int I = i >> 1, In = (i & 1) ? I + 1 : I - 1;
    const T e0 = line[(int64_t)I * stride];
    const T e1 = (In >= 0 && In < n) ? line[(int64_t)In * stride] : -e0;
    return T(0.75) * e0 + T(0.25) * e1;
}

// cell-centred cubic Lagrange interpolation: (-5, 35, 105, -7)/128 on I-2..I+1
// for the fine cell at I - H/4, mirrored for I + H/4
template <typename T>
__device__ __forceinline__ T cubic_at(const T* __restrict__ line, int64_t stride, int n, int i)
{
    const int I = i >> 1;
    if ((i & 1) == 0)
        return (T(-5) * odd_at(line, stride, n, I - 2) + T(35) * odd_at(line, stride, n, I - 1) +
                T(105) * odd_at(line, stride, n, I) - T(7) * odd_at(line, stride, n, I + 1)) /
               T(128);
    return (T(-7) * odd_at(line, stride, n, I - 1) + T(105) * odd_at(line, stride, n, I) +
            T(35) * odd_at(line, stride, n, I + 1) - T(5) * odd_at(line, stride, n, I + 2)) /
           T(128);
}

// block-wide sum of two values; result valid in thread 0
__device__ __forceinline__ void block_sum2(double& a, double& b)
{
    __shared__ double sa[kBlock / 64], sb[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) { sa[w] = a; sb[w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = sa[0]; b = sb[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) { a += sa[k]; b += sb[k]; }
    }
}

// ------------------------------------------------------------------------
// Coefficient field k = exp(Z) at the faces of one grid for a list of samples.
// Z = sum_{m<Mx, n<My} C_mn cos(pi m x) cos(pi n y); C is built per block from
// xi and the field spec; the double sum is evaluated as a product of the
// per-column cosine table and the per-row partial sums D_m(y) = sum_n C_mn cos(pi n y).
// ------------------------------------------------------------------------
constexpr int kFieldTI = 64, kFieldTJ = 16;

__device__ __forceinline__ double cospi_ratio(int64_t num, int64_t den)
{
    // cos(pi num/den) with the argument reduced exactly modulo 2
    int64_t r = num % (2 * den);
    if (r < 0) r += 2 * den;
    return cospi((double)r / (double)den);
}

__global__ void __launch_bounds__(kBlock)
k_field(FieldArgs A, const int32_t* __restrict__ samples, const SampleBase* __restrict__ bases,
        const double* __restrict__ xi, double* __restrict__ KX, double* __restrict__ KY,
        float* __restrict__ KX32, float* __restrict__ KY32)
{
    extern __shared__ double sm[];
    const int Mx = A.Mx, My = A.My;
    double* C = sm;                              // Mx*My
    double* cx = C + Mx * My;                    // Mx*(kFieldTI)
    double* D = cx + Mx * kFieldTI;              // Mx*kFieldTJ
    const int s = samples[blockIdx.y];
    const SampleBase sb = bases[s];
    const double* xs = xi + (int64_t)s * A.n_terms;

    // coefficient matrix of this sample
    for (int idx = threadIdx.x; idx < Mx * My; idx += blockDim.x) C[idx] = 0.0;
    __syncthreads();
    if (A.kind == 0) {
        if (threadIdx.x == 0)
            for (int t = 0; t < A.cos.n; ++t) C[A.cos.a[t] * My + A.cos.b[t]] += A.cos.amp[t] * xs[t];
    } else {
        for (int idx = threadIdx.x; idx < Mx * My; idx += blockDim.x) {
            const int m = idx / My, n = idx % My;
            const double nm = m == 0 ? 1.0 : sqrt(2.0), nn = n == 0 ? 1.0 : sqrt(2.0);
            C[idx] = A.sigma * sqrt(A.lamx[m] * A.lamy[n]) * nm * nn * xs[m * My + n];
        }
    }
    __syncthreads();

    // this block's tile of faces
    const int kind = A.kind_faces;                 // 0: x-faces, 1: y-faces
    const int nx = A.nx, ny = A.ny;
    const int fw = kind == 0 ? nx + 1 : nx;        // faces per row
    const int fh = kind == 0 ? ny : ny + 1;        // rows of faces
    const int tiles_x = (fw + kFieldTI - 1) / kFieldTI;
    const int i0 = (blockIdx.x % tiles_x) * kFieldTI, j0 = (blockIdx.x / tiles_x) * kFieldTJ;
    // x position of face column i: i/nx (x-faces) or (2i+1)/(2nx) (y-faces)
    for (int idx = threadIdx.x; idx < Mx * kFieldTI; idx += blockDim.x) {
        const int m = idx / kFieldTI, li = idx % kFieldTI, i = i0 + li;
        cx[idx] = kind == 0 ? cospi_ratio((int64_t)m * i, nx) : cospi_ratio((int64_t)m * (2 * i + 1), 2 * nx);
    }
    // D_m(y_j) for the tile's rows; y position (2j+1)/(2ny) (x-faces) or j/ny (y-faces)
    for (int idx = threadIdx.x; idx < Mx * kFieldTJ; idx += blockDim.x) {
        const int m = idx / kFieldTJ, lj = idx % kFieldTJ, j = j0 + lj;
        double d = 0.0;
        for (int n = 0; n < My; ++n) {
            const double cy = kind == 0 ? cospi_ratio((int64_t)n * (2 * j + 1), 2 * ny) : cospi_ratio((int64_t)n * j, ny);
            d += C[m * My + n] * cy;
        }
        D[idx] = d;
    }
    __syncthreads();
    const int64_t base = kind == 0 ? sb.fx + xface_off(A.c, sb.Q, A.p, A.q) : sb.fy + yface_off(A.c, sb.Q, A.p, A.q);
    double* out = kind == 0 ? KX : KY;
    float* out32 = kind == 0 ? KX32 : KY32;
    for (int idx = threadIdx.x; idx < kFieldTI * kFieldTJ; idx += blockDim.x) {
        const int li = idx % kFieldTI, lj = idx / kFieldTI;
        const int i = i0 + li, j = j0 + lj;
        if (i >= fw || j >= fh) continue;
        double z = 0.0;
        for (int m = 0; m < Mx; ++m) z += cx[m * kFieldTI + li] * D[m * kFieldTJ + lj];
        const double k = exp(z);
        const int64_t o = base + (int64_t)j * fw + i;
        out[o] = k;
        if (out32) out32[o] = (float)k;
    }
}

// ------------------------------------------------------------------------
// Face-mean coefficients (MSG_FACE_MEAN): every face of grid (p,q) of a
// sample takes the mean of the finest grid's face values lying on it, summed
// in order along the face.  An x-face (i,j) lies on the finest x-face column
// i 2^(P-p) and spans its rows j 2^(Q-q) .. (j+1) 2^(Q-q) - 1; a y-face (i,j)
// lies on the finest y-face row j 2^(Q-q) and spans its columns
// i 2^(P-p) .. (i+1) 2^(P-p) - 1.  The finest grid itself is left as
// synthesised.  One thread per output face; blockIdx.y is the sample of the
// list.  The reads of neighbouring threads are strided by 2^(P-p) elements
// (x-faces) or contiguous runs (y-faces), served mostly from L2: the finest
// grid of a sample is a few hundred KB.
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_face_mean(int c, int p, int q, int kind_faces, const int32_t* __restrict__ samples,
            const SampleBase* __restrict__ bases, double* __restrict__ KX, double* __restrict__ KY,
            float* __restrict__ KX32, float* __restrict__ KY32)
{
    const SampleBase sb = bases[samples[blockIdx.y]];
    if (p == sb.P && q == sb.Q) return;
    const int nx = c << p, ny = c << q, nxF = c << sb.P;
    const int rx = 1 << (sb.P - p), ry = 1 << (sb.Q - q);
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (kind_faces == 0) {
        if (f >= (int64_t)(nx + 1) * ny) return;
        const int i = (int)(f % (nx + 1)), j = (int)(f / (nx + 1));
        const double* src = KX + sb.fx + xface_off(c, sb.Q, sb.P, sb.Q) + (int64_t)j * ry * (nxF + 1) + (int64_t)i * rx;
        double sum = 0.0;
        for (int t = 0; t < ry; ++t) sum += src[(int64_t)t * (nxF + 1)];
        const double k = sum / (double)ry;
        const int64_t o = sb.fx + xface_off(c, sb.Q, p, q) + f;
        KX[o] = k;
        if (KX32) KX32[o] = (float)k;
    } else {
        if (f >= (int64_t)nx * (ny + 1)) return;
        const int i = (int)(f % nx), j = (int)(f / nx);
        const double* src = KY + sb.fy + yface_off(c, sb.Q, sb.P, sb.Q) + (int64_t)j * ry * nxF + (int64_t)i * rx;
        double sum = 0.0;
        for (int t = 0; t < rx; ++t) sum += src[t];
        const double k = sum / (double)rx;
        const int64_t o = sb.fy + yface_off(c, sb.Q, p, q) + f;
        KY[o] = k;
        if (KY32) KY32[o] = (float)k;
    }
}

// ------------------------------------------------------------------------
// Standard normal KL coefficients drawn on the device: xi[s][t] is normal t
// of the stream (seed, id[s]): Philox4x64-10 at counter (t/4, id, 0, 0),
// key (seed, kKlKey); words (0,1) give normals 4n (rho cos) and 4n+1
// (rho sin) by the Box-Muller transform, words (2,3) normals 4n+2 and 4n+3.
// One thread per group of four normals.
// ------------------------------------------------------------------------
constexpr uint64_t kKlKey = 0x4B4C2D7869ull;

__global__ void __launch_bounds__(kBlock)
k_kl_xi(int S, int n_terms, uint64_t seed, const int64_t* __restrict__ ids, double* __restrict__ xi)
{
    const int groups = (n_terms + 3) / 4;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)S * groups) return;
    const int s = (int)(g / groups), n = (int)(g % groups);
    uint64_t w[4] = {(uint64_t)n, (uint64_t)ids[s], 0, 0};
    philox4x64_10(w, seed, kKlKey);
    double* out = xi + (int64_t)s * n_terms;
    for (int h = 0; h < 2; ++h) {
        const double rho = sqrt(-2.0 * log(uniform52(w[2 * h])));
        double sn, cs;
        sincos(2.0 * M_PI * uniform52(w[2 * h + 1]), &sn, &cs);
        const int t = 4 * n + 2 * h;
        if (t < n_terms) out[t] = rho * cs;
        if (t + 1 < n_terms) out[t + 1] = rho * sn;
    }
}

// ------------------------------------------------------------------------
// Coarsest grid: dense Cholesky of A^(0,0) (c^2 unknowns) once per sample,
// assembled column by column from the stencil, then the inverse from the
// factor (L^-T L^-1, one column per lane); one wavefront per sample.  Every
// coarsest solve of the cycles is then one small matrix-vector product.
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(64)
k_chol(int S, int c, const SampleBase* __restrict__ bases, const double* __restrict__ KX,
       const double* __restrict__ KY, double* __restrict__ chol)
{
    extern __shared__ double A[];                 // n*n factor, then n*n inverse columns
    const int s = blockIdx.x;
    if (s >= S) return;
    const int n = c * c;
    const SampleBase sb = bases[s];
    const double* kx = KX + sb.fx;                 // grid (0,0) is first in the sample
    const double* ky = KY + sb.fy;
    const double ih2 = (double)c * c;
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) A[idx] = 0.0;
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const int i = k % c, j = k / c;
        const Stencil<double> w = stencil_at(kx, ky, c, c, i, j, ih2, ih2);
        A[k * n + k] = w.wW + w.wE + w.wS + w.wN;
        if (i > 0) A[(k - 1) * n + k] = -w.wW;
        if (i < c - 1) A[(k + 1) * n + k] = -w.wE;
        if (j > 0) A[(k - c) * n + k] = -w.wS;
        if (j < c - 1) A[(k + c) * n + k] = -w.wN;
    }
    __syncthreads();
    double* L = chol + (int64_t)s * n * n;
    // lower factor overwrites A column by column
    for (int j = 0; j < n; ++j) {
        if (threadIdx.x == 0) {
            double d = A[j * n + j];
            for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
            A[j * n + j] = sqrt(d);
        }
        __syncthreads();
        for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) {
            double t = A[i * n + j];
            for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = t / A[j * n + j];
        }
        __syncthreads();
    }
    // column j of A^-1: L y = e_j, then L^T x = y (lane j, n <= 64)
    double* X = A + n * n;
    const int j = threadIdx.x;
    if (j < n) {
        for (int i = 0; i < n; ++i) {
            double t = i == j ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) t -= A[i * n + k] * X[k * n + j];
            X[i * n + j] = t / A[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double t = X[i * n + j];
            for (int k = i + 1; k < n; ++k) t -= A[k * n + i] * X[k * n + j];
            X[i * n + j] = t / A[i * n + i];
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) L[idx] = X[idx];
}

// ------------------------------------------------------------------------
// Helpers shared by the level kernels: block -> (problem, grid, tile)
// ------------------------------------------------------------------------
struct Where {
    int k;       // problem
    int gi;      // grid inside the launch
    int t;       // tile inside the grid
};

// Blocks are dealt to the 8 XCDs round-robin (block i on XCD i mod 8); the
// grid is padded to a multiple of 8 and block i works on logical block
// (i mod 8) * (n/8) + i/8, so each XCD gets one contiguous run of tiles and
// neighbouring tiles share that XCD's L2.  Padding blocks get k = -1.
__device__ __forceinline__ Where locate(const KLevel& L)
{
    Where w;
    const int per = gridDim.x >> 3;
    const int b = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (b >= L.nblocks) { w.k = -1; w.gi = 0; w.t = 0; return w; }
    w.k = b / L.ntiles;
    int t = b - w.k * L.ntiles;
    int gi = 0;
    while (gi + 1 < L.ngrids && t >= L.g[gi + 1].tile0) ++gi;
    w.gi = gi;
    w.t = t - L.g[gi].tile0;
    return w;
}

// ------------------------------------------------------------------------
// Red-black Gauss-Seidel (Section 2: nu1 = nu2 = 2 sweeps), NS sweeps fused
// per pass: the tile's iterate plus a halo of 2*NS cells sits in LDS; each
// half-sweep updates one colour on a region that shrinks by one cell, so the
// tile interior ends exactly as NS global red-then-black sweeps would leave it.
// The pass reads Vin and writes Vout (a different buffer): neighbouring tiles
// read their halos from Vin while this tile writes, so an in-place update
// would race.
// ------------------------------------------------------------------------
//
// NS = 0 copies the tile (a pass that keeps the buffer parity of a level).
//
// CORR: the pass starts from v + omega * (coarse-grid correction of eq.
// interpolation), computed while the tile and its halo are loaded, so the
// correction needs no pass of its own (same arithmetic as k_prolong).
template <typename T>
__device__ __forceinline__ T correction_at(const KGrid& G, const KProb& pr, int c, const T* __restrict__ Vc,
                                           const T* __restrict__ kx, const T* __restrict__ ky, int i, int j)
{
    const int nx = G.nx, ny = G.ny;
    const bool hx = G.aoff_x >= 0, hy = G.aoff_y >= 0;
    T ex = T(0), ey = T(0);
    if (hx) ex = linear_at(Vc + pr.arena_base + G.aoff_x + (int64_t)j * (nx / 2), (int64_t)1, nx / 2, i);
    if (hy) ey = linear_at(Vc + pr.arena_base + G.aoff_y + i, (int64_t)nx, ny / 2, j);
    if (hx && hy) {
        const T ka = kappa_x_at(kx, ky, nx, ny, i, j, T(nx) * T(nx), T(ny) * T(ny));
        return ka * ex + (T(1) - ka) * ey;
    }
    return hx ? ex : ey;
}

//
// CORR and RS with NS = 4: the post-smoothing pass of one W-cycle visit of a
// level and the pre-smoothing pass of the next visit, which follow each
// other with nothing in between, as one pass (the restricted values go to
// the coarse iterate buffer that does not hold the correction being read).
//
// RS (with NS = 2, no correction): the pre-smoothing pass also forms the
// residual of its tile's cells and restricts it into level l-1 (eq.
// restriction), so the iterate, right-hand side and conductances are not read
// again.  The halo is one cell wider, so that the cells just outside the tile
// hold their final values too.  A coarse grid with one parent gets its
// right-hand side and a zero iterate here; one with two parents gets the
// x-parent's half in its right-hand side and the y-parent's in its iterate,
// and k_restrict_combine adds them.
template <typename T, int NS, bool CORR, int NT, bool RS = false>
__global__ void __launch_bounds__(NT)
k_rbgs(KLevel L, const KProb* __restrict__ probs, const int32_t* __restrict__ active, int c,
       const T* __restrict__ Vin, T* __restrict__ Vout, const T* __restrict__ B, const T* __restrict__ KX,
       const T* __restrict__ KY, const T* __restrict__ Vc, T omega, T* __restrict__ Bco, T* __restrict__ Vco)
{
    constexpr int H = 2 * NS + (RS ? 1 : 0);
    extern __shared__ __align__(16) unsigned char smem_rb[];
    T* sv = reinterpret_cast<T*>(smem_rb);
    const Where w = locate(L);
    if (w.k < 0 || !active[w.k]) return;
    const KGrid& G = L.g[w.gi];
    const KProb pr = probs[w.k];
    const int nx = G.nx, ny = G.ny, tw = G.tw, th = G.th;
    const int i0 = (w.t % G.tiles_x) * tw, j0 = (w.t / G.tiles_x) * th;
    const T* v = Vin + pr.arena_base + G.aoff;
    T* vout = Vout + pr.arena_base + G.aoff;
    const T* b = B + pr.arena_base + G.aoff;
    const T* kx = KX + pr.fx_base + xface_off(c, pr.Qs, G.p, G.q);
    const T* ky = KY + pr.fy_base + yface_off(c, pr.Qs, G.p, G.q);
    const T ihx2 = T(nx) * T(nx), ihy2 = T(ny) * T(ny);
    // a direction in which the tile spans the whole grid has no neighbouring
    // tile: one cell of zeros (the wall) is all the halo it needs
    const int Hx = G.tiles_x > 1 ? H : 1, Hy = th < ny ? H : 1;
    const int RW = tw + 2 * Hx, RH = th + 2 * Hy;

    for (int idx = threadIdx.x; idx < RW * RH; idx += NT) {
        const int i = i0 - Hx + idx % RW, j = j0 - Hy + idx / RW;
        T x = T(0);
        if (i >= 0 && i < nx && j >= 0 && j < ny) {
            x = v[(int64_t)j * nx + i];
            if (CORR) x += omega * correction_at(G, pr, c, Vc, kx, ky, i, j);
        }
        sv[idx] = x;
    }
    __syncthreads();
    for (int s = 0; s < NS; ++s) {
        for (int colour = 0; colour < 2; ++colour) {
            const int e = H - 1 - 2 * s - colour;            // extent of this half-sweep beyond the tile
            const int xa = max(i0 - e, 0), xb = min(i0 + tw + e, nx);
            const int ya = max(j0 - e, 0), yb = min(j0 + th + e, ny);
            const int EW = xb - xa, EH = yb - ya, slots = (EW + 1) >> 1;
            for (int idx = threadIdx.x; idx < slots * EH; idx += NT) {
                const int lj = idx / slots, j = ya + lj;
                const int li = 2 * (idx - lj * slots) + ((colour - xa - j) & 1);
                if (li >= EW) continue;
                const int i = xa + li;
                const Stencil<T> st = stencil_at(kx, ky, nx, ny, i, j, ihx2, ihy2);
                const int r = (j - j0 + Hy) * RW + (i - i0 + Hx);
                sv[r] = gs_update(st, b[(int64_t)j * nx + i], sv[r - 1], sv[r + 1], sv[r - RW], sv[r + RW]);
            }
            __syncthreads();
        }
    }
    for (int idx = threadIdx.x; idx < tw * th; idx += NT) {
        const int li = idx % tw, lj = idx / tw, i = i0 + li, j = j0 + lj;
        if (i < nx && j < ny) vout[(int64_t)j * nx + i] = sv[(lj + Hy) * RW + li + Hx];
    }
    if constexpr (RS) {
        // b - A v at a cell of the tile, from the swept tile in LDS (the
        // arithmetic of residual_at)
        auto tres = [&](int i, int j) -> T {
            const Stencil<T> st = stencil_at(kx, ky, nx, ny, i, j, ihx2, ihy2);
            const int r = (j - j0 + Hy) * RW + (i - i0 + Hx);
            const T u = sv[r];
            const T uW = i > 0 ? sv[r - 1] : T(0);
            const T uE = i < nx - 1 ? sv[r + 1] : T(0);
            const T uS = j > 0 ? sv[r - RW] : T(0);
            const T uN = j < ny - 1 ? sv[r + RW] : T(0);
            return b[(int64_t)j * nx + i] - (st.wW * (u - uW) + st.wE * (u - uE) + st.wS * (u - uS) + st.wN * (u - uN));
        };
        // each iteration takes a block of 2 x 2 fine cells (2 x 1 or 1 x 2 when
        // the grid restricts in one direction only) and computes each
        // residual once for both children
        const int iw = min(tw, nx - i0), jh = min(th, ny - j0);
        const bool hx = G.aoff_x >= 0, hy = G.aoff_y >= 0;
        const int bw = hx ? 2 : 1, bh = hy ? 2 : 1, nbx = iw / bw, nby = jh / bh;
        const int nxc = nx >> 1;
        for (int idx = threadIdx.x; idx < nbx * nby; idx += NT) {
            const int by = idx / nbx, i = i0 + (idx - by * nbx) * bw, j = j0 + by * bh;
            const T r00 = tres(i, j);
            const T r10 = hx ? tres(i + 1, j) : T(0);
            const T r01 = hy ? tres(i, j + 1) : T(0);
            const T r11 = (hx && hy) ? tres(i + 1, j + 1) : T(0);
            if (hx) {                               // into (p-1,q): pairs of columns
                const int64_t cx = pr.arena_base + G.aoff_x + (int64_t)j * nxc + (i >> 1);
                Bco[cx] = T(0.5) * (r00 + r10);
                if (!(G.rflags & 1)) Vco[cx] = T(0);
                if (hy) {
                    Bco[cx + nxc] = T(0.5) * (r01 + r11);
                    if (!(G.rflags & 1)) Vco[cx + nxc] = T(0);
                }
            }
            if (hy) {                               // into (p,q-1): pairs of rows
                const int64_t cy = pr.arena_base + G.aoff_y + (int64_t)(j >> 1) * nx + i;
                const T ry0 = T(0.5) * (r00 + r01);
                if (G.rflags & 2) {
                    Vco[cy] = ry0;
                } else {
                    Bco[cy] = ry0;
                    Vco[cy] = T(0);
                }
                if (hx) {
                    const T ry1 = T(0.5) * (r10 + r11);
                    if (G.rflags & 2) {
                        Vco[cy + 1] = ry1;
                    } else {
                        Bco[cy + 1] = ry1;
                        Vco[cy + 1] = T(0);
                    }
                }
            }
        }
    }
}

// One colour of a red-black half-sweep over whole grids in global memory,
// in place (cells of one colour have no neighbour of that colour), one
// thread per cell.  Used only by the split-sweep debug mode, which runs the
// fused passes as their separate steps to check them bit for bit.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_rb_colour(KLevel L, const KProb* __restrict__ probs, const int32_t* __restrict__ active, int c, int colour,
            T* __restrict__ V, const T* __restrict__ B, const T* __restrict__ KX, const T* __restrict__ KY)
{
    const Where w = locate(L);
    if (w.k < 0 || !active[w.k]) return;
    const KGrid& G = L.g[w.gi];
    const KProb pr = probs[w.k];
    const int64_t cell = (int64_t)w.t * blockDim.x + threadIdx.x;
    const int nx = G.nx, ny = G.ny;
    if (cell >= (int64_t)nx * ny) return;
    const int i = (int)(cell % nx), j = (int)(cell / nx);
    if (((i + j) & 1) != colour) return;
    T* v = V + pr.arena_base + G.aoff;
    const T* kx = KX + pr.fx_base + xface_off(c, pr.Qs, G.p, G.q);
    const T* ky = KY + pr.fy_base + yface_off(c, pr.Qs, G.p, G.q);
    const Stencil<T> st = stencil_at(kx, ky, nx, ny, i, j, T(nx) * T(nx), T(ny) * T(ny));
    const T vW = i > 0 ? v[cell - 1] : T(0);
    const T vE = i < nx - 1 ? v[cell + 1] : T(0);
    const T vS = j > 0 ? v[cell - nx] : T(0);
    const T vN = j < ny - 1 ? v[cell + nx] : T(0);
    v[cell] = gs_update(st, B[pr.arena_base + G.aoff + cell], vW, vE, vS, vN);
}

// The coarse grids with two parents after a restricting pass: b = average
// of the two halves (eq. restriction), iterate zeroed.  L is the coarse level
// with its parents' offsets.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_restrict_combine(KLevel L, const KProb* __restrict__ probs, const int32_t* __restrict__ active, T* __restrict__ Vc,
                   T* __restrict__ B)
{
    const Where w = locate(L);
    if (w.k < 0 || !active[w.k]) return;
    const KGrid& G = L.g[w.gi];
    if (G.aoff_x < 0 || G.aoff_y < 0) return;
    const KProb pr = probs[w.k];
    const int64_t cell = (int64_t)w.t * blockDim.x + threadIdx.x;
    if (cell >= (int64_t)G.nx * G.ny) return;
    const int64_t a = pr.arena_base + G.aoff + cell;
    B[a] = T(0.5) * B[a] + T(0.5) * Vc[a];
    Vc[a] = T(0);
}

// ------------------------------------------------------------------------
// Residual and restriction (eq. restriction): coarse b = average of the
// x-restricted residual of (p+1,q) and the y-restricted residual of (p,q+1),
// one-sided where only one exists; the coarse iterate is zeroed.  With
// RHS = true the fine quantity is the right-hand side itself (F-cycle).
// One thread per coarse cell; a block takes consecutive cells of one grid.
// ------------------------------------------------------------------------
template <typename T, bool RHS>
__global__ void __launch_bounds__(kBlock)
k_restrict(KLevel L, const KProb* __restrict__ probs, const int32_t* __restrict__ active, int c,
           const T* __restrict__ Vf, T* __restrict__ Vc, T* __restrict__ B, const T* __restrict__ KX,
           const T* __restrict__ KY)
{
    const Where w = locate(L);
    if (w.k < 0 || (active && !active[w.k])) return;
    const KGrid& G = L.g[w.gi];
    const KProb pr = probs[w.k];
    const int64_t cell = (int64_t)w.t * blockDim.x + threadIdx.x;
    const int nx = G.nx, ny = G.ny;
    if (cell >= (int64_t)nx * ny) return;
    const int I = (int)(cell % nx), J = (int)(cell / nx);
    T rx = T(0), ry = T(0);
    const bool hx = G.aoff_x >= 0, hy = G.aoff_y >= 0;
    if (hx) {                                   // fine grid (p+1,q): 2nx x ny
        const int fnx = 2 * nx;
        const T* vf = Vf + pr.arena_base + G.aoff_x;
        const T* bf = B + pr.arena_base + G.aoff_x;
        if (RHS) {
            rx = T(0.5) * (bf[(int64_t)J * fnx + 2 * I] + bf[(int64_t)J * fnx + 2 * I + 1]);
        } else {
            const T* kx = KX + pr.fx_base + xface_off(c, pr.Qs, G.p + 1, G.q);
            const T* ky = KY + pr.fy_base + yface_off(c, pr.Qs, G.p + 1, G.q);
            const T ihx2 = T(fnx) * T(fnx), ihy2 = T(ny) * T(ny);
            rx = T(0.5) * (residual_at(vf, bf, kx, ky, fnx, ny, 2 * I, J, ihx2, ihy2) +
                           residual_at(vf, bf, kx, ky, fnx, ny, 2 * I + 1, J, ihx2, ihy2));
        }
    }
    if (hy) {                                   // fine grid (p,q+1): nx x 2ny
        const int fny = 2 * ny;
        const T* vf = Vf + pr.arena_base + G.aoff_y;
        const T* bf = B + pr.arena_base + G.aoff_y;
        if (RHS) {
            ry = T(0.5) * (bf[(int64_t)(2 * J) * nx + I] + bf[(int64_t)(2 * J + 1) * nx + I]);
        } else {
            const T* kx = KX + pr.fx_base + xface_off(c, pr.Qs, G.p, G.q + 1);
            const T* ky = KY + pr.fy_base + yface_off(c, pr.Qs, G.p, G.q + 1);
            const T ihx2 = T(nx) * T(nx), ihy2 = T(fny) * T(fny);
            ry = T(0.5) * (residual_at(vf, bf, kx, ky, nx, fny, I, 2 * J, ihx2, ihy2) +
                           residual_at(vf, bf, kx, ky, nx, fny, I, 2 * J + 1, ihx2, ihy2));
        }
    }
    const T bc = (hx && hy) ? T(0.5) * rx + T(0.5) * ry : (hx ? rx : ry);
    B[pr.arena_base + G.aoff + cell] = bc;
    if (!RHS) Vc[pr.arena_base + G.aoff + cell] = T(0);
}

// ------------------------------------------------------------------------
// Coarse-grid correction (eq. interpolation): v += omega (kappa_x P_x e^(p-1,q)
// + kappa_y P_y e^(p,q-1)), one-sided on q = 0 (P_x only) and p = 0 (P_y only).
// ------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_prolong(KLevel L, const KProb* __restrict__ probs, const int32_t* __restrict__ active, int c, T omega,
          const T* __restrict__ Vc, T* __restrict__ Vf, const T* __restrict__ KX, const T* __restrict__ KY)
{
    const Where w = locate(L);
    if (w.k < 0 || !active[w.k]) return;
    const KGrid& G = L.g[w.gi];
    const KProb pr = probs[w.k];
    const int64_t cell = (int64_t)w.t * blockDim.x + threadIdx.x;
    const int nx = G.nx, ny = G.ny;
    if (cell >= (int64_t)nx * ny) return;
    const int i = (int)(cell % nx), j = (int)(cell / nx);
    const bool hx = G.aoff_x >= 0, hy = G.aoff_y >= 0;
    T ex = T(0), ey = T(0);
    if (hx) ex = linear_at(Vc + pr.arena_base + G.aoff_x + (int64_t)j * (nx / 2), (int64_t)1, nx / 2, i);
    if (hy) ey = linear_at(Vc + pr.arena_base + G.aoff_y + i, (int64_t)nx, ny / 2, j);
    T corr;
    if (hx && hy) {
        const T* kx = KX + pr.fx_base + xface_off(c, pr.Qs, G.p, G.q);
        const T* ky = KY + pr.fy_base + yface_off(c, pr.Qs, G.p, G.q);
        const T ka = kappa_x_at(kx, ky, nx, ny, i, j, T(nx) * T(nx), T(ny) * T(ny));
        corr = ka * ex + (T(1) - ka) * ey;
    } else {
        corr = hx ? ex : ey;
    }
    Vf[pr.arena_base + G.aoff + cell] += omega * corr;
}

// ------------------------------------------------------------------------
// Nested iteration (Algorithm MSG F-cycle): the initial iterate of each
// problem's finest grid is the weighted cubic interpolation of the solutions
// of (p-1,q) and (p,q-1) returned by the previous level; its right-hand side
// is copied from the restricted right-hand side pyramid.
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_fmg(KLevel L, const KProb* __restrict__ probs, const int32_t* __restrict__ active, int c,
      double* __restrict__ V, double* __restrict__ B, const double* __restrict__ U,
      const double* __restrict__ BP, const double* __restrict__ KX, const double* __restrict__ KY)
{
    const Where w = locate(L);
    if (w.k < 0 || !active[w.k]) return;
    const KGrid& G = L.g[w.gi];
    const KProb pr = probs[w.k];
    const int64_t cell = (int64_t)w.t * blockDim.x + threadIdx.x;
    const int nx = G.nx, ny = G.ny;
    if (cell >= (int64_t)nx * ny) return;
    const int i = (int)(cell % nx), j = (int)(cell / nx);
    const bool hx = G.p > 0, hy = G.q > 0;
    double ex = 0.0, ey = 0.0;
    if (hx) ex = cubic_at(U + pr.cell_base + cell_off(c, pr.Qs, G.p - 1, G.q) + (int64_t)j * (nx / 2), (int64_t)1, nx / 2, i);
    if (hy) ey = cubic_at(U + pr.cell_base + cell_off(c, pr.Qs, G.p, G.q - 1) + i, (int64_t)nx, ny / 2, j);
    double v0;
    if (hx && hy) {
        const double* kx = KX + pr.fx_base + xface_off(c, pr.Qs, G.p, G.q);
        const double* ky = KY + pr.fy_base + yface_off(c, pr.Qs, G.p, G.q);
        const double ka = kappa_x_at(kx, ky, nx, ny, i, j, (double)nx * nx, (double)ny * ny);
        v0 = ka * ex + (1.0 - ka) * ey;
    } else if (hx || hy) {
        v0 = hx ? ex : ey;
    } else {
        v0 = 0.0;                                  // the coarsest grid starts from zero
    }
    V[pr.arena_base + G.aoff + cell] = v0;
    B[pr.arena_base + G.aoff + cell] = BP[pr.cell_base + cell_off(c, pr.Qs, G.p, G.q) + cell];
}

// ------------------------------------------------------------------------
// Residual norm of each problem's finest grid in FP64: per block partial sums
// of r^2 and b^2 (fixed order, so a problem's result does not depend on the
// rest of the batch).  In mixed precision the FP64 residual is also handed to
// the FP32 inner cycle as its right-hand side, with a zero FP32 iterate.
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_resnorm(KLevel L, const KProb* __restrict__ probs, const int32_t* __restrict__ active, int c,
          const double* __restrict__ V, const double* __restrict__ B, const double* __restrict__ KX,
          const double* __restrict__ KY, double* __restrict__ part, float* __restrict__ V32,
          float* __restrict__ B32)
{
    const Where w = locate(L);
    if (w.k < 0 || !active[w.k]) return;
    const KGrid& G = L.g[w.gi];
    const KProb pr = probs[w.k];
    const int64_t cell = (int64_t)w.t * blockDim.x + threadIdx.x;
    const int nx = G.nx, ny = G.ny;
    double rr = 0.0, bb = 0.0;
    if (cell < (int64_t)nx * ny) {
        const int i = (int)(cell % nx), j = (int)(cell / nx);
        const double* v = V + pr.arena_base + G.aoff;
        const double* b = B + pr.arena_base + G.aoff;
        const double* kx = KX + pr.fx_base + xface_off(c, pr.Qs, G.p, G.q);
        const double* ky = KY + pr.fy_base + yface_off(c, pr.Qs, G.p, G.q);
        const double r = residual_at(v, b, kx, ky, nx, ny, i, j, (double)nx * nx, (double)ny * ny);
        rr = r * r;
        bb = b[cell] * b[cell];
        if (B32) {
            B32[pr.arena_base + G.aoff + cell] = (float)r;
            V32[pr.arena_base + G.aoff + cell] = 0.0f;
        }
    }
    block_sum2(rr, bb);
    if (threadIdx.x == 0) {
        part[2 * (pr.part_base + w.t)] = rr;
        part[2 * (pr.part_base + w.t) + 1] = bb;
    }
}

// Convergence decision per problem (adaptive nu0 of Section 2): one wavefront
// sums the partials; converged problems and non-finite ones stop cycling.
__global__ void __launch_bounds__(64)
k_converge(int K, int ntiles, const KProb* __restrict__ probs, int32_t* __restrict__ active,
           int32_t* __restrict__ pcycles, int32_t* __restrict__ dead_level, int32_t* __restrict__ status,
           const double* __restrict__ part, double tol, int max_cycles, int level, int32_t* __restrict__ n_active)
{
    const int k = blockIdx.x;
    if (k >= K || !active[k]) return;
    const KProb pr = probs[k];
    double rr = 0.0, bb = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += 64) {
        rr += part[2 * (pr.part_base + t)];
        bb += part[2 * (pr.part_base + t) + 1];
    }
    for (int off = 32; off > 0; off >>= 1) {
        rr += __shfl_down(rr, off, 64);
        bb += __shfl_down(bb, off, 64);
    }
    if (threadIdx.x != 0) return;
    const double rn = sqrt(rr), bn = sqrt(bb);
    if (!isfinite(rn) || !isfinite(bn)) {
        active[k] = 0;
        atomicMax(&status[pr.sample], (int)MSG_ST_NONFINITE);
        atomicMin(&dead_level[pr.sample], level);
        return;
    }
    if (rn <= tol * bn) { active[k] = 0; return; }
    if (pcycles[k] >= max_cycles) {
        active[k] = 0;
        atomicMax(&status[pr.sample], (int)MSG_ST_MAXITER);
        return;
    }
    pcycles[k] += 1;                 // one more cycle is about to run
    atomicAdd(n_active, 1);
}

// start of an F-cycle level: every problem cycles unless its sample already
// went non-finite on a lower level
__global__ void __launch_bounds__(kBlock)
k_activate(int K, const KProb* __restrict__ probs, const int32_t* __restrict__ dead_level, int level,
           int32_t* __restrict__ active, int32_t* __restrict__ pcycles)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    active[k] = dead_level[probs[k].sample] > level ? 1 : 0;
    pcycles[k] = 0;
}

// mixed precision: the FP64 iterate takes the FP32 correction
__global__ void __launch_bounds__(kBlock)
k_ir_update(KLevel L, const KProb* __restrict__ probs, const int32_t* __restrict__ active,
            double* __restrict__ V, const float* __restrict__ V32)
{
    const Where w = locate(L);
    if (w.k < 0 || !active[w.k]) return;
    const KGrid& G = L.g[w.gi];
    const KProb pr = probs[w.k];
    const int64_t cell = (int64_t)w.t * blockDim.x + threadIdx.x;
    if (cell >= (int64_t)G.nx * G.ny) return;
    V[pr.arena_base + G.aoff + cell] += (double)V32[pr.arena_base + G.aoff + cell];
}

// ------------------------------------------------------------------------
// Snapshot at the end of an F-cycle level: the problem's finest-grid iterate
// becomes the returned solution of grid (p,q) (NaN when its sample went
// non-finite on this level or below), with partial sums for Q = mean of u.
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_snapshot(KLevel L, const KProb* __restrict__ probs, const int32_t* __restrict__ dead_level, int level, int c,
           const double* __restrict__ V, double* __restrict__ U, double* __restrict__ part)
{
    const Where w = locate(L);
    if (w.k < 0) return;
    const KGrid& G = L.g[w.gi];
    const KProb pr = probs[w.k];
    const int64_t cell = (int64_t)w.t * blockDim.x + threadIdx.x;
    const bool dead = dead_level[pr.sample] <= level;
    double u = 0.0, zero = 0.0;
    if (cell < (int64_t)G.nx * G.ny) {
        u = dead ? __longlong_as_double(0x7ff8000000000000LL) : V[pr.arena_base + G.aoff + cell];
        U[pr.cell_base + cell_off(c, pr.Qs, G.p, G.q) + cell] = u;
    }
    block_sum2(u, zero);
    if (threadIdx.x == 0) part[2 * (pr.part_base + w.t)] = u;
}

__global__ void __launch_bounds__(64)
k_qreduce(int K, int ntiles, int64_t cells, const KProb* __restrict__ probs, const int32_t* __restrict__ pcycles,
          const int64_t* __restrict__ grid_base, const double* __restrict__ part, double* __restrict__ q_out,
          int32_t* __restrict__ cycles_out)
{
    const int k = blockIdx.x;
    if (k >= K) return;
    const KProb pr = probs[k];
    double s = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += 64) s += part[2 * (pr.part_base + t)];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (threadIdx.x == 0) {
        q_out[grid_base[pr.sample] + pr.grid_index] = s / (double)cells;
        if (cycles_out) cycles_out[grid_base[pr.sample] + pr.grid_index] = pcycles[k];
    }
}

// right-hand side on each sample's finest grid: h = 1, or the caller's values
__global__ void __launch_bounds__(kBlock)
k_rhs_top(KLevel L, const KProb* __restrict__ probs, double* __restrict__ BP, const double* __restrict__ rhs,
          const int64_t* __restrict__ rhs_base)
{
    const Where w = locate(L);
    if (w.k < 0) return;
    const KGrid& G = L.g[w.gi];
    const KProb pr = probs[w.k];
    const int64_t cell = (int64_t)w.t * blockDim.x + threadIdx.x;
    if (cell >= (int64_t)G.nx * G.ny) return;
    BP[pr.arena_base + G.aoff + cell] = rhs ? rhs[rhs_base[pr.sample] + cell] : 1.0;
}

// ------------------------------------------------------------------------
// Tail: the mu-cycles of levels 0..top of one problem run inside one
// wavefront, with every grid of those levels (iterate, right-hand side and
// face coefficients) held in LDS; the coarsest grid is solved with the
// sample's FP64 inverse.  The top level's iterate and right-hand
// side come from the arena and the iterate goes back there.  A single wave
// per problem keeps every phase barrier local to the wave, and many small
// workgroups per CU hide the latency of the short dependent phases.
// ------------------------------------------------------------------------
// (i,j) of linear cell index idx on a grid of width nx (log2 width sh, or -1)
__device__ __forceinline__ void cell_ij(int idx, int nx, int sh, int& i, int& j)
{
    if (sh >= 0) { j = idx >> sh; i = idx & (nx - 1); }
    else { j = idx / nx; i = idx - j * nx; }
}

// One grid of a tail level as seen by one lane: its shape and where its
// arrays sit in LDS (closed forms of the level layout, see KTail).
struct TGrid {
    int p, q, nx, ny, sh;      // sh = log2(nx) or -1
    int v, b, x, y;            // LDS element offsets
};

__device__ __forceinline__ TGrid tgrid(const KTail& TL, const KTailLevel& L, int lev, int g)
{
    TGrid G;
    G.p = L.pmin + g;
    G.q = lev - G.p;
    G.nx = TL.c << G.p;
    G.ny = TL.c << G.q;
    G.sh = TL.lc >= 0 ? TL.lc + G.p : -1;
    G.v = L.v0 + g * L.cells;
    G.b = L.b0 + g * L.cells;
    const int qmax = lev - L.pmin;
    G.x = L.x0 + g * L.cells + TL.c * ((2 << qmax) - (2 << qmax >> g));
    G.y = L.y0 + g * L.cells + (TL.c << L.pmin) * ((1 << g) - 1);
    return G;
}

// slot -> (grid, index inside the grid) when every grid owns `per` slots
__device__ __forceinline__ void split_slot(int sl, int per, int psh, int& g, int& local)
{
    if (psh >= 0) { g = sl >> psh; local = sl & (per - 1); }
    else { g = sl / per; local = sl - g * per; }
}

// b - A v at (i,j) from LDS, conductances already scaled by 1/h^2 with the
// wall faces doubled
// The four neighbours of (i,j) read without branches: each load goes to a
// valid cell of the grid (the centre where the neighbour is a wall) and the
// wall value zero is selected afterwards, so all loads issue together.
template <typename T>
struct Nbr {
    T W, E, S, N;
};

template <typename T>
__device__ __forceinline__ Nbr<T> neighbours(const T* v, int off, int i, int j, int nx, int ny)
{
    const bool w = i > 0, e = i < nx - 1, s = j > 0, n = j < ny - 1;
    const T xW = v[w ? off - 1 : off], xE = v[e ? off + 1 : off];
    const T xS = v[s ? off - nx : off], xN = v[n ? off + nx : off];
    return Nbr<T>{w ? xW : T(0), e ? xE : T(0), s ? xS : T(0), n ? xN : T(0)};
}

// (a neighbour beyond a wall is read from the zero element z of the tail)
template <typename T>
__device__ __forceinline__ T tresid(const T* sm, const TGrid& G, int i, int j, int z)
{
    const int off = G.v + j * G.nx + i;
    const T cW = sm[G.x + j * (G.nx + 1) + i], cE = sm[G.x + j * (G.nx + 1) + i + 1];
    const T cS = sm[G.y + j * G.nx + i], cN = sm[G.y + (j + 1) * G.nx + i];
    const T u = sm[off], bb = sm[G.b + j * G.nx + i];
    const T xW = sm[i > 0 ? off - 1 : z], xE = sm[i < G.nx - 1 ? off + 1 : z];
    const T xS = sm[j > 0 ? off - G.nx : z], xN = sm[j < G.ny - 1 ? off + G.nx : z];
    return bb - (cW * (u - xW) + cE * (u - xE) + cS * (u - xS) + cN * (u - xN));
}

// linear interpolation of eq. interpolation along a line of LDS (32-bit
// indexing; the arithmetic of linear_at)
template <typename T>
__device__ __forceinline__ T linear_lds(const T* line, int stride, int n, int i)
{
    const int I = i >> 1, In = (i & 1) ? I + 1 : I - 1;
    const T e0 = line[I * stride];
    const T e1 = (In >= 0 && In < n) ? line[In * stride] : -e0;
    return T(0.75) * e0 + T(0.25) * e1;
}

// kappa of eq. interpolation at cell (i,j) of a tail grid with both coarse
// children (the weights of tail_prolong)
template <typename T>
__device__ __forceinline__ T tail_kappa(const T* sm, const TGrid& G, int i, int j)
{
    const T cW = sm[G.x + j * (G.nx + 1) + i], cE = sm[G.x + j * (G.nx + 1) + i + 1];
    const T cS = sm[G.y + j * G.nx + i], cN = sm[G.y + (j + 1) * G.nx + i];
    T lx = (i == 0 ? cW : T(2) * cW) + (i == G.nx - 1 ? cE : T(2) * cE);
    T ly = (j == 0 ? cS : T(2) * cS) + (j == G.ny - 1 ? cN : T(2) * cN);
    if (j == 0) lx += cS;
    if (j == G.ny - 1) lx += cN;
    if (i == 0) ly += cW;
    if (i == G.nx - 1) ly += cE;
    const T a = lx * lx, b = ly * ly;
    return a / (a + b);
}

// the face conductances of every tail grid of problem pr, k/h^2 with the wall
// faces doubled, written to dst in the tail layout (LDS or the prepared image)
template <typename T, int NT>
__device__ __forceinline__ void tail_faces(const KTail& TL, const KProb& pr, int c, const T* __restrict__ KX,
                                           const T* __restrict__ KY, T* dst)
{
    for (int lev = 0; lev <= TL.top; ++lev) {
        const KTailLevel L = TL.lvl[lev];
        for (int g = 0; g < L.ng; ++g) {
            const TGrid G = tgrid(TL, L, lev, g);
            const T* kx = KX + pr.fx_base + xface_off(c, pr.Qs, G.p, G.q);
            const T* ky = KY + pr.fy_base + yface_off(c, pr.Qs, G.p, G.q);
            const T ihx2 = T(G.nx) * T(G.nx), ihy2 = T(G.ny) * T(G.ny);
            const int nfx = (G.nx + 1) * G.ny, nfy = G.nx * (G.ny + 1);
            for (int idx = threadIdx.x; idx < nfx; idx += NT) {
                const int i = idx % (G.nx + 1);
                const T w = kx[idx] * ihx2;
                dst[G.x + idx] = (i == 0 || i == G.nx) ? T(2) * w : w;
            }
            for (int idx = threadIdx.x; idx < nfy; idx += NT) {
                const int j = idx / G.nx;
                const T w = ky[idx] * ihy2;
                dst[G.y + idx] = (j == 0 || j == G.ny) ? T(2) * w : w;
            }
        }
    }
}

// The conductance image of the tail of every problem of a class, prepared
// once per F-cycle stage: pack[k*nstat ...] is what k_tail copies into LDS.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_tail_pack(const KTail* __restrict__ table, const KProb* __restrict__ probs, int c, const T* __restrict__ KX,
            const T* __restrict__ KY, T* __restrict__ pack)
{
    const KTail& TL = *table;
    const int k = blockIdx.x;
    tail_faces<T, kBlock>(TL, probs[k], c, KX, KY, pack + (int64_t)k * TL.nstat);
}

// every grid of level lev, `sweeps` red-then-black sweeps; one colour of all
// the level's grids is spread over the lanes
// The slot table of a tail (see KTail::slots), from the same decoding the
// smoother uses without it.  One workgroup per tail.
__global__ void __launch_bounds__(kBlock)
k_tail_slots(const KTail* __restrict__ table, int4* __restrict__ out)
{
    const KTail& TL = *table;
    for (int lev = 0; lev <= TL.top; ++lev) {
        const KTailLevel L = TL.lvl[lev];
        const int per = L.cells >> 1;
        const int psh = L.csh >= 0 ? L.csh - 1 : -1;
        for (int sl = threadIdx.x; sl < per * L.ng; sl += blockDim.x) {
            int g, local, k, j;
            split_slot(sl, per, psh, g, local);
            const TGrid G = tgrid(TL, L, lev, g);
            cell_ij(local, G.nx >> 1, G.sh >= 1 ? G.sh - 1 : -1, k, j);
            const int bits = G.nx | ((j & 1) << 16) | ((k == 0) << 17) | ((2 * k + 2 == G.nx) << 18) | ((j == 0) << 19) |
                             ((j == G.ny - 1) << 20);
            out[TL.slot_off[lev] + sl] = make_int4(G.v + j * G.nx + 2 * k, G.x + j * (G.nx + 1) + 2 * k,
                                                   G.y + j * G.nx + 2 * k, bits);
        }
    }
}

// Barrier between the phases of the on-chip tail.  A workgroup of one
// wavefront needs no hardware barrier: its LDS instructions are executed in
// program order, so a later read by any lane sees an earlier write.  Only
// the compiler must keep LDS accesses on their side of the phase boundary.
template <int NT>
__device__ __forceinline__ void tail_sync()
{
    if constexpr (NT == 64) {
        __builtin_amdgcn_wave_barrier();
        asm volatile("" ::: "memory");
    } else {
        __syncthreads();
    }
}

// every grid of level lev, `sweeps` red-then-black sweeps from the slot
// table: the same updates, in the same arithmetic, as the decoding loop below
// slot-table entries are read through a global (not flat) pointer: a flat
// load in flight also holds the LDS counter, so every LDS read after it would
// wait for the table as well
typedef int SlotV __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) SlotV* SlotPtr;

// one red-black update of the cell at `off` (this colour's cell of its pair);
// a neighbour beyond a wall is read from the zero element z
template <typename T>
__device__ __forceinline__ T tail_cell_update(const T* sm, SlotV e, int d, int db, T inv, int z)
{
    const int nx = e.w & 0xffff;
    const int off = e.x + d, fx = e.y + d, fy = e.z + d;
    const T cW = sm[fx], cE = sm[fx + 1];
    const T cS = sm[fy], cN = sm[fy + nx];
    const T bb = sm[off + db];
    const bool w = !((e.w >> 17) & 1) || d, ea = !((e.w >> 18) & 1) || !d;
    const bool so = !((e.w >> 19) & 1), no = !((e.w >> 20) & 1);
    const T xW = sm[w ? off - 1 : z], xE = sm[ea ? off + 1 : z];
    const T xS = sm[so ? off - nx : z], xN = sm[no ? off + nx : z];
    return (bb + cW * xW + cE * xE + cS * xS + cN * xN) * inv;
}

template <typename T>
__device__ __forceinline__ T tail_inv_diag(const T* sm, SlotV e, int d)
{
    const int nx = e.w & 0xffff;
    const int fx = e.y + d, fy = e.z + d;
    return T(1) / (sm[fx] + sm[fx + 1] + sm[fy] + sm[fy + nx]);
}

// Levels of at most R slots per thread: the entries and the reciprocal
// diagonals of both cells of every slot stay in registers for all sweeps
// (the conductances do not change while smoothing), so the table is read
// once and each cell divides once per call.
template <typename T, int NT, int R>
__device__ __forceinline__ void tail_smooth_regs(T* sm, SlotPtr tab, int total, int db, int z, int sweeps)
{
    SlotV e[R];
    T i0[R], i1[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int sl = (int)threadIdx.x + r * NT;
        e[r] = sl < total ? tab[sl] : SlotV{0, 0, 0, 0};
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        i0[r] = T(0);
        i1[r] = T(0);
        if ((int)threadIdx.x + r * NT < total) {
            i0[r] = tail_inv_diag(sm, e[r], 0);
            i1[r] = tail_inv_diag(sm, e[r], 1);
        }
    }
    for (int s = 0; s < sweeps; ++s)
        for (int colour = 0; colour < 2; ++colour) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if ((int)threadIdx.x + r * NT < total) {
                    // FP64, several slots per lane: the entry passes through an
                    // empty asm statement so that the cell addresses are formed
                    // again at each half-sweep rather than held for all R slots
                    // (about 50 registers fewer: more room for the smoother's
                    // wavefronts beside the tail; FP32 tails measured faster
                    // with the addresses held)
                    int ex = e[r].x, ey = e[r].y, ez = e[r].z, ew = e[r].w;
                    if constexpr (R > 1 && sizeof(T) == 8) asm volatile("" : "+v"(ex), "+v"(ey), "+v"(ez), "+v"(ew));
                    const SlotV ee = SlotV{ex, ey, ez, ew};
                    const int d = (colour + (ee.w >> 16)) & 1;
                    sm[ee.x + d] = tail_cell_update(sm, ee, d, db, d ? i1[r] : i0[r], z);
                }
            }
            tail_sync<NT>();
        }
}

// The small levels of a tail (one slot per lane at most) are smoothed many
// times per launch: a W-cycle visits level l 2^(top-l) times.  Their slot
// entry and the reciprocal diagonals of its two cells are formed once, when
// the launch starts (the conductances stay fixed for the whole launch), and
// held in registers; each smoothing call then only sweeps.  Same arithmetic
// as tail_smooth_regs.  Levels 1..kTailRegLevels at most.

template <typename T>
struct TailRegLevel {
    SlotV e;
    T i0, i1;
    bool on;                                        // this lane owns a slot of the level
    // restriction into level lev-1, lane = coarse cell of that level: the
    // slots (lanes) of level lev holding its x-parent pair and its y-parent
    // pairs, with flags (see tail_restrict_reg), and its LDS iterate offset
    int rrec, rdst;
    bool ron;                                       // this lane has a coarse cell
};

template <typename T, int NT>
__device__ __forceinline__ TailRegLevel<T> tail_reg_level(const KTail& TL, const T* sm, int lev)
{
    TailRegLevel<T> R;
    R.e = SlotV{0, 0, 0, 0};
    R.i0 = T(0);
    R.i1 = T(0);
    R.on = false;
    if (lev > TL.top || lev > TL.reg_levels) return R;
    const KTailLevel L = TL.lvl[lev];
    const int total = (L.cells >> 1) * L.ng;
    if (total <= NT && (int)threadIdx.x < total) {
        R.e = ((SlotPtr)(TL.slots + TL.slot_off[lev]))[threadIdx.x];
        R.i0 = tail_inv_diag(sm, R.e, 0);
        R.i1 = tail_inv_diag(sm, R.e, 1);
        R.on = true;
    }
    R.rrec = 0;
    R.rdst = 0;
    R.ron = false;
    // coarse cell (I,J) of grid G = (p,q) on level lev-1: its x-parent
    // (p+1,q) holds fine cells (2I,J), (2I+1,J), the pair of slot I of row J;
    // its y-parent (p,q+1) holds (I,2J) and (I,2J+1), cells I&1 of the pairs
    // of slot I>>1 in rows 2J and 2J+1 (nx/2 slots apart)
    const KTailLevel C = TL.lvl[lev - 1];
    const int per = L.cells >> 1, ctotal = C.cells * C.ng;
    if (total <= 64 && ctotal <= 64 && (int)threadIdx.x < ctotal) {
        int g, off, I, J;
        split_slot((int)threadIdx.x, C.cells, C.csh, g, off);
        const TGrid G = tgrid(TL, C, lev - 1, g);
        cell_ij(off, G.nx, G.sh, I, J);
        const bool hx = G.p + 1 <= TL.pc, hy = G.q + 1 <= TL.qc;
        const int sx = hx ? (G.p + 1 - L.pmin) * per + J * G.nx + I : 0;
        const int sy = hy ? (G.p - L.pmin) * per + J * G.nx + (I >> 1) : 0;
        const int step = hy ? G.nx >> 1 : 0;
        R.rrec = sx | (sy << 7) | (step << 14) | ((int)hx << 21) | ((int)hy << 22) | ((I & 1) << 23);
        R.rdst = G.v + off;
        R.ron = true;
    }
    return R;
}

// b - A v at cell d of a slot's pair, from LDS (the arithmetic of tresid)
template <typename T>
__device__ __forceinline__ T tail_pair_resid(const T* sm, SlotV e, int d, int db, int z)
{
    const int nx = e.w & 0xffff;
    const int off = e.x + d, fx = e.y + d, fy = e.z + d;
    const T cW = sm[fx], cE = sm[fx + 1];
    const T cS = sm[fy], cN = sm[fy + nx];
    const T u = sm[off], bb = sm[off + db];
    const bool w = !((e.w >> 17) & 1) || d, ea = !((e.w >> 18) & 1) || !d;
    const bool so = !((e.w >> 19) & 1), no = !((e.w >> 20) & 1);
    const T xW = sm[w ? off - 1 : z], xE = sm[ea ? off + 1 : z];
    const T xS = sm[so ? off - nx : z], xN = sm[no ? off + nx : z];
    return bb - (cW * (u - xW) + cE * (u - xE) + cS * (u - xS) + cN * (u - xN));
}

template <typename T, int NT>
__device__ __forceinline__ void tail_sweeps_reg(T* sm, const TailRegLevel<T>& R, int db, int z, int sweeps)
{
    // the entry passes through an empty asm statement, so the compiler forms
    // the cell addresses from it at each call instead of keeping those of
    // every level live for the whole launch (which took the kernel from 161
    // to 226 registers and left no room on a SIMD for the smoother's
    // wavefronts running beside the tail: slower on the overlapped step)
    int ex = R.e.x, ey = R.e.y, ez = R.e.z, ew = R.e.w;
    asm volatile("" : "+v"(ex), "+v"(ey), "+v"(ez), "+v"(ew));
    const SlotV e = SlotV{ex, ey, ez, ew};
    for (int s = 0; s < sweeps; ++s)
        for (int colour = 0; colour < 2; ++colour) {
            if (R.on) {
                const int d = (colour + (e.w >> 16)) & 1;
                sm[e.x + d] = tail_cell_update(sm, e, d, db, d ? R.i1 : R.i0, z);
            }
            tail_sync<NT>();
        }
}

template <typename T>
struct TailRegs {
    TailRegLevel<T> r1, r2, r3;
};

template <typename T, int NT>
__device__ __forceinline__ void tail_smooth_table(const KTail& TL, T* sm, int lev, int sweeps)
{
    const KTailLevel L = TL.lvl[lev];
    const int total = (L.cells >> 1) * L.ng;
    const int db = L.b0 - L.v0;                     // right-hand side of a cell, relative to its iterate
    const SlotPtr tab = (SlotPtr)(TL.slots + TL.slot_off[lev]);
    if (total <= NT) {
        tail_smooth_regs<T, NT, 1>(sm, tab, total, db, TL.zero, sweeps);
        return;
    }
    if (total <= 4 * NT) {
        tail_smooth_regs<T, NT, 4>(sm, tab, total, db, TL.zero, sweeps);
        return;
    }
    for (int s = 0; s < sweeps; ++s)
        for (int colour = 0; colour < 2; ++colour) {
            int sl = threadIdx.x;
            SlotV e = sl < total ? tab[sl] : SlotV{0, 0, 0, 0};
            for (; sl < total; sl += NT) {
                const SlotV en = sl + NT < total ? tab[sl + NT] : e;   // the next entry, in flight meanwhile
                const int d = (colour + (e.w >> 16)) & 1;
                sm[e.x + d] = tail_cell_update(sm, e, d, db, tail_inv_diag(sm, e, d), TL.zero);
                e = en;
            }
            tail_sync<NT>();
        }
}

template <typename T, int NT>
__device__ __forceinline__ void tail_smooth(const KTail& TL, T* sm, int lev, int sweeps, const TailRegs<T>& RG,
                                            bool regs)
{
    const KTailLevel L = TL.lvl[lev];
    const bool pairs = !(TL.c & 1);                 // nx even on every grid
    if (regs && lev <= TL.reg_levels && (L.cells >> 1) * L.ng <= NT) {
        const int db = L.b0 - L.v0;
        if (lev == 1) { tail_sweeps_reg<T, NT>(sm, RG.r1, db, TL.zero, sweeps); return; }
        if (lev == 2) { tail_sweeps_reg<T, NT>(sm, RG.r2, db, TL.zero, sweeps); return; }
        if (lev == 3) { tail_sweeps_reg<T, NT>(sm, RG.r3, db, TL.zero, sweeps); return; }
    }
    if (pairs && TL.slots) {
        tail_smooth_table<T, NT>(TL, sm, lev, sweeps);
        return;
    }
    const int per = pairs ? L.cells >> 1 : L.cells;
    const int psh = L.csh >= 0 ? (pairs ? L.csh - 1 : L.csh) : -1;
    const int total = per * L.ng;
    for (int s = 0; s < sweeps; ++s)
        for (int colour = 0; colour < 2; ++colour) {
            for (int sl = threadIdx.x; sl < total; sl += NT) {
                int g, local;
                split_slot(sl, per, psh, g, local);
                const TGrid G = tgrid(TL, L, lev, g);
                int i, j;
                if (pairs) {
                    int k;
                    cell_ij(local, G.nx >> 1, G.sh >= 1 ? G.sh - 1 : -1, k, j);
                    i = 2 * k + ((colour + j) & 1);     // pair k of row j holds this colour's cell
                } else {
                    cell_ij(local, G.nx, G.sh, i, j);
                    if (((i + j) & 1) != colour) continue;
                }
                T* v = sm + G.v;
                const int off = j * G.nx + i;
                const T cW = sm[G.x + j * (G.nx + 1) + i], cE = sm[G.x + j * (G.nx + 1) + i + 1];
                const T cS = sm[G.y + j * G.nx + i], cN = sm[G.y + (j + 1) * G.nx + i];
                const T bb = sm[G.b + off];
                const Nbr<T> nb = neighbours(v, off, i, j, G.nx, G.ny);
                v[off] = (bb + cW * nb.W + cE * nb.E + cS * nb.S + cN * nb.N) / (cW + cE + cS + cN);
            }
            tail_sync<NT>();
        }
}

// tail_restrict on a level whose pairs and coarse cells fit one per lane of
// the first wavefront: each lane forms the residuals of its own fine pair
// from its slot entry, and each coarse cell gathers its parents' residuals
// from the lanes holding them.  Same arithmetic as tail_restrict.
template <typename T, int NT>
__device__ __forceinline__ void tail_restrict_reg(const KTail& TL, T* sm, int lev, const TailRegLevel<T>& R)
{
    const KTailLevel F = TL.lvl[lev], C = TL.lvl[lev - 1];
    const int dbf = F.b0 - F.v0, dbc = C.b0 - C.v0;
    int ex = R.e.x, ey = R.e.y, ez = R.e.z, ew = R.e.w;
    asm volatile("" : "+v"(ex), "+v"(ey), "+v"(ez), "+v"(ew));
    const SlotV e = SlotV{ex, ey, ez, ew};
    T r0 = T(0), r1 = T(0);
    if (R.on) {
        r0 = tail_pair_resid(sm, e, 0, dbf, TL.zero);
        r1 = tail_pair_resid(sm, e, 1, dbf, TL.zero);
    }
    const T rxp = T(0.5) * (r0 + r1);               // the pair's cells restricted in x
    const int rec = R.rrec;
    const int sx = rec & 127, sy = (rec >> 7) & 127, step = (rec >> 14) & 127;
    const T gx = __shfl(rxp, sx, 64);
    const T a0 = __shfl(r0, sy, 64), a1 = __shfl(r1, sy, 64);
    const T c0 = __shfl(r0, sy + step, 64), c1 = __shfl(r1, sy + step, 64);
    if (R.ron) {
        const bool hx = (rec >> 21) & 1, hy = (rec >> 22) & 1, odd = (rec >> 23) & 1;
        const T rx = gx;
        const T ry = T(0.5) * ((odd ? a1 : a0) + (odd ? c1 : c0));
        sm[R.rdst + dbc] = (hx && hy) ? T(0.5) * rx + T(0.5) * ry : (hx ? rx : ry);
        sm[R.rdst] = T(0);
    }
    tail_sync<NT>();
}

// residual of level lev restricted to level lev-1 (eq. restriction); the
// coarse iterate is zeroed
template <typename T, int NT>
__device__ __forceinline__ void tail_restrict(const KTail& TL, T* sm, int lev, const TailRegs<T>& RG, bool regs)
{
    if (regs && lev <= TL.reg_levels) {
        const KTailLevel F = TL.lvl[lev], C = TL.lvl[lev - 1];
        if ((F.cells >> 1) * F.ng <= 64 && C.cells * C.ng <= 64) {
            if (lev == 1) { tail_restrict_reg<T, NT>(TL, sm, 1, RG.r1); return; }
            if (lev == 2) { tail_restrict_reg<T, NT>(TL, sm, 2, RG.r2); return; }
            if (lev == 3) { tail_restrict_reg<T, NT>(TL, sm, 3, RG.r3); return; }
        }
    }
    const KTailLevel C = TL.lvl[lev - 1], F = TL.lvl[lev];
    const int total = C.cells * C.ng;
    for (int sl = threadIdx.x; sl < total; sl += NT) {
        int g, off;
        split_slot(sl, C.cells, C.csh, g, off);
        const TGrid G = tgrid(TL, C, lev - 1, g);
        int I, J;
        cell_ij(off, G.nx, G.sh, I, J);
        const bool hx = G.p + 1 <= TL.pc, hy = G.q + 1 <= TL.qc;
        T rx = T(0), ry = T(0);
        if (hx) {
            const TGrid P = tgrid(TL, F, lev, G.p + 1 - F.pmin);
            rx = T(0.5) * (tresid(sm, P, 2 * I, J, TL.zero) + tresid(sm, P, 2 * I + 1, J, TL.zero));
        }
        if (hy) {
            const TGrid P = tgrid(TL, F, lev, G.p - F.pmin);
            ry = T(0.5) * (tresid(sm, P, I, 2 * J, TL.zero) + tresid(sm, P, I, 2 * J + 1, TL.zero));
        }
        sm[G.b + off] = (hx && hy) ? T(0.5) * rx + T(0.5) * ry : (hx ? rx : ry);
        sm[G.v + off] = T(0);
    }
    tail_sync<NT>();
}

// eq. interpolation on level lev from level lev-1, weights from the scaled
// conductances: an interior face contributes 2c to lambda, a wall face c
template <typename T, int NT>
__device__ __forceinline__ void tail_prolong(const KTail& TL, T* sm, int lev, T omega)
{
    const KTailLevel F = TL.lvl[lev], C = TL.lvl[lev - 1];
    const int total = F.cells * F.ng;
    for (int sl = threadIdx.x; sl < total; sl += NT) {
        int g, off;
        split_slot(sl, F.cells, F.csh, g, off);
        const TGrid G = tgrid(TL, F, lev, g);
        int i, j;
        cell_ij(off, G.nx, G.sh, i, j);
        const bool hx = G.p > 0, hy = G.q > 0;
        T ex = T(0), ey = T(0);
        if (hx) {
            const TGrid X = tgrid(TL, C, lev - 1, G.p - 1 - C.pmin);
            ex = linear_lds(sm + X.v + j * (G.nx / 2), 1, G.nx / 2, i);
        }
        if (hy) {
            const TGrid Y = tgrid(TL, C, lev - 1, G.p - C.pmin);
            ey = linear_lds(sm + Y.v + i, G.nx, G.ny / 2, j);
        }
        T corr;
        if (hx && hy) {
            const T ka = tail_kappa(sm, G, i, j);
            corr = ka * ex + (T(1) - ka) * ey;
        } else {
            corr = hx ? ex : ey;
        }
        sm[G.v + off] += omega * corr;
    }
    tail_sync<NT>();
}

// v^(0,0) = (A^(0,0))^-1 b^(0,0) in FP64, lane k computing unknown k (c^2 <= 64)
// from the sample's inverse
template <typename T, int NT>
__device__ __forceinline__ void tail_coarse(const KTail& TL, T* sm, const double* Ai, int n)
{
    const KTailLevel L0 = TL.lvl[0];
    const int k = threadIdx.x;
    if (k < n) {
        const T* b = sm + L0.b0;
        double x = 0.0;
        for (int j = 0; j < n; ++j) x += Ai[k * n + j] * (double)b[j];
        sm[L0.v0 + k] = (T)x;
    }
    tail_sync<NT>();
}

// count mu-cycles on the tail's top level; the recursion is unrolled with
// the cycles still to run on each level kept two bits per level in a register
template <typename T, int NT>
__device__ __forceinline__ void tail_cycles(const KTail& TL, T* sm, const double* Lc, int n0, int mu, int nu1,
                                            int nu2, T omega, int count, const TailRegs<T>& RG, bool regs)
{
    uint64_t left = 0;
    auto get = [&](int l) { return (int)((left >> (2 * l)) & 3u); };
    auto set = [&](int l, int v) { left = (left & ~((uint64_t)3 << (2 * l))) | ((uint64_t)v << (2 * l)); };
    int lev = TL.top;
    set(lev, count);
    bool down = true;
    // The coarsest solve overwrites v^(0,0) from b^(0,0) alone, and nothing
    // changes b^(0,0) between the mu calls of one visit of level 1 (nor
    // between cycles when level 0 is the top): the repeated solves would
    // write the same bits, so only the first after a restriction runs.
    bool solved0 = false;
    for (;;) {
        if (down) {
            if (lev == 0) {
                if (!solved0) tail_coarse<T, NT>(TL, sm, Lc, n0);
                solved0 = true;
                down = false;
                continue;
            }
            tail_smooth<T, NT>(TL, sm, lev, nu1, RG, regs);
            tail_restrict<T, NT>(TL, sm, lev, RG, regs);
            --lev;
            if (lev == 0) solved0 = false;
            set(lev, mu);
        } else {
            // one cycle on level lev just finished
            const int l = get(lev) - 1;
            set(lev, l);
            if (l > 0) { down = true; continue; }
            if (lev == TL.top) break;
            ++lev;
            tail_prolong<T, NT>(TL, sm, lev, omega);
            tail_smooth<T, NT>(TL, sm, lev, nu2, RG, regs);
        }
    }
}

// ||b - A v||_2^2 and ||b||_2^2 of the (single) top grid over the workgroup
template <typename T, int NT>
__device__ __forceinline__ void tail_norms(const KTail& TL, T* sm, double& rr, double& bb)
{
    __shared__ double red[2][NT / 64];
    const KTailLevel L = TL.lvl[TL.top];
    const TGrid G = tgrid(TL, L, TL.top, 0);
    rr = 0.0;
    bb = 0.0;
    for (int off = threadIdx.x; off < L.cells; off += NT) {
        int i, j;
        cell_ij(off, G.nx, G.sh, i, j);
        const double r = (double)tresid(sm, G, i, j, TL.zero);
        const double b = (double)sm[G.b + off];
        rr += r * r;
        bb += b * b;
    }
    for (int o = 32; o > 0; o >>= 1) {
        rr += __shfl_xor(rr, o, 64);
        bb += __shfl_xor(bb, o, 64);
    }
    if (NT > 64) {
        if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = rr; red[1][threadIdx.x >> 6] = bb; }
        tail_sync<NT>();
        rr = red[0][0];
        bb = red[1][0];
        for (int w = 1; w < NT / 64; ++w) { rr += red[0][w]; bb += red[1][w]; }
        tail_sync<NT>();
    }
}

// count > 0: that many mu-cycles on the top level.  count < 0: the whole
// adaptive loop of one F-cycle level (Section 2: cycle until ||r|| <= tol ||b||,
// checked before every cycle) for problems whose rectangle fits in LDS,
// updating cycle counts, status and the non-finite level like k_converge.
// Block b works on problem b of the launch, problem kbase + b of the stage's
// table, with class descriptor tables[cls[b]] (cls given: several classes in
// one launch, -1 = skip) or tables[tidx]; with `pack`, its conductance image
// is image (kbase + b - first) of its class, at the class's pack_off.
template <typename T, int NT>
__global__ void __launch_bounds__(NT)
k_tail(const KTail* __restrict__ tables, const int32_t* __restrict__ cls, int tidx, int kbase,
       const KProb* __restrict__ probs, const int32_t* __restrict__ active, int c, int mu, int nu1,
       int nu2, T omega, int count, int combine, T* __restrict__ V, T* __restrict__ B, const T* __restrict__ KX,
       const T* __restrict__ KY, const T* __restrict__ pack, const double* __restrict__ chol, TailSolve ad)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int k = blockIdx.x;
    const int t = cls ? cls[k] : tidx;
    if (t < 0 || !active[k]) return;
    const KTail& TL = tables[t];
    T* sm = reinterpret_cast<T*>(smem);
    double* Lc = reinterpret_cast<double*>(smem + TL.chol_off);
    const KProb pr = probs[k];
    const int n0 = c * c;
    // stage in: the face conductances of every grid (the prepared image, or
    // computed here from the coefficients), the top level's iterates and
    // right-hand sides, the coarsest inverse
    if (pack) {
        const uint4* src =
            reinterpret_cast<const uint4*>(pack + TL.pack_off + (int64_t)(kbase + k - TL.first) * TL.nstat);
        uint4* dst = reinterpret_cast<uint4*>(sm);
        const int n16 = TL.nstat * (int)sizeof(T) / 16;
        for (int idx = threadIdx.x; idx < n16; idx += NT) dst[idx] = src[idx];
    } else {
        tail_faces<T, NT>(TL, pr, c, KX, KY, sm);
    }
    {
        // combine: the top level was just restricted by the restricting
        // pre-smoothing pass, which leaves a grid with two parents holding
        // the x-parent's half in its right-hand side and the y-parent's in
        // its iterate; they are averaged here (eq. restriction) and the
        // iterate starts from zero
        const KTailLevel L = TL.lvl[TL.top];
        for (int g = 0; g < L.ng; ++g) {
            const int64_t a = pr.arena_base + TL.top_aoff[g];
            const int v0 = L.v0 + g * L.cells, b0 = L.b0 + g * L.cells;
            const int p = L.pmin + g, q = TL.top - p;
            if (combine && p + 1 <= TL.pc && q + 1 <= TL.qc) {
                for (int idx = threadIdx.x; idx < L.cells; idx += NT) {
                    sm[b0 + idx] = T(0.5) * B[a + idx] + T(0.5) * V[a + idx];
                    sm[v0 + idx] = T(0);
                }
            } else {
                for (int idx = threadIdx.x; idx < L.cells; idx += NT) {
                    sm[v0 + idx] = V[a + idx];
                    sm[b0 + idx] = B[a + idx];
                }
            }
        }
    }
    for (int idx = threadIdx.x; idx < n0 * n0; idx += NT) Lc[idx] = chol[(int64_t)pr.sample * n0 * n0 + idx];
    if (threadIdx.x == 0) sm[TL.zero] = T(0);
    __syncthreads();
    const bool use_regs = TL.reg_levels > 0 && TL.slots && !(TL.c & 1);
    TailRegs<T> RG;
    RG.r1 = tail_reg_level<T, NT>(TL, sm, use_regs ? 1 : kMaxTailLevels);
    RG.r2 = tail_reg_level<T, NT>(TL, sm, use_regs ? 2 : kMaxTailLevels);
    RG.r3 = tail_reg_level<T, NT>(TL, sm, use_regs ? 3 : kMaxTailLevels);

    if (count > 0) {
        tail_cycles<T, NT>(TL, sm, Lc, n0, mu, nu1, nu2, omega, count, RG, use_regs);
    } else {
        int ncyc = ad.pcycles[k];                // cycles already run on this level
        for (;;) {
            double rr, bb;
            tail_norms<T, NT>(TL, sm, rr, bb);
            const double rn = sqrt(rr), bn = sqrt(bb);
            if (!isfinite(rn) || !isfinite(bn)) {
                if (threadIdx.x == 0) {
                    atomicMax(&ad.status[pr.sample], (int)MSG_ST_NONFINITE);
                    atomicMin(&ad.dead_level[pr.sample], ad.level);
                }
                break;
            }
            if (rn <= ad.tol * bn) break;
            if (ncyc >= ad.max_cycles) {
                if (threadIdx.x == 0) atomicMax(&ad.status[pr.sample], (int)MSG_ST_MAXITER);
                break;
            }
            tail_cycles<T, NT>(TL, sm, Lc, n0, mu, nu1, nu2, omega, 1, RG, use_regs);
            ++ncyc;
        }
        if (threadIdx.x == 0) ad.pcycles[k] = ncyc;
    }
    // stage out the top level's iterates
    {
        const KTailLevel L = TL.lvl[TL.top];
        for (int g = 0; g < L.ng; ++g) {
            const int64_t a = pr.arena_base + TL.top_aoff[g];
            const int v0 = L.v0 + g * L.cells;
            for (int idx = threadIdx.x; idx < L.cells; idx += NT) V[a + idx] = sm[v0 + idx];
        }
    }
}

// ------------------------------------------------------------------------
// Multi-index differences (Section 3), one thread per (sample, grid)
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_delta_q(int S, const int32_t* __restrict__ PQ, const int64_t* __restrict__ gbase, const double* __restrict__ q,
          double* __restrict__ dq)
{
    const int s = blockIdx.y;
    if (s >= S) return;
    const int P = PQ[2 * s], Q = PQ[2 * s + 1];
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (P + 1) * (Q + 1)) return;
    const int p = g / (Q + 1), r = g % (Q + 1);
    const double* qs = q + gbase[s];
    double d = qs[g];
    if (p > 0) d -= qs[g - (Q + 1)];
    if (r > 0) d -= qs[g - 1];
    if (p > 0 && r > 0) d += qs[g - (Q + 1) - 1];
    dq[gbase[s] + g] = d;
}

// ------------------------------------------------------------------------
// Plain cycles from zero (the convergence-factor comparison of Section 2):
// the finest grid's iterate zero and right-hand side h = 1 or the caller's
// values (sample-major, one finest grid after the other); standard
// multigrid's transfers between grid (p,q) and (p-1,q-1), the products of the
// one-directional cell-centred operators; the coarsest solve by the sample's
// inverse; residual-norm ratios per problem.
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_plain_init(KLevel L, const KProb* __restrict__ probs, const double* __restrict__ rhs, double* __restrict__ V,
             double* __restrict__ B)
{
    const Where w = locate(L);
    if (w.k < 0) return;
    const KGrid& G = L.g[w.gi];
    const KProb pr = probs[w.k];
    const int64_t n = (int64_t)G.nx * G.ny;
    const int64_t cell = (int64_t)w.t * blockDim.x + threadIdx.x;
    if (cell >= n) return;
    V[pr.arena_base + G.aoff + cell] = 0.0;
    B[pr.arena_base + G.aoff + cell] = rhs ? rhs[(int64_t)pr.sample * n + cell] : 1.0;
}

// coarse grid (I,J) of G takes the average of the residuals of the four fine
// cells of grid (p+1,q+1) at aoff_x; its iterate is zeroed
__global__ void __launch_bounds__(kBlock)
k_restrict2d(KLevel L, const KProb* __restrict__ probs, const int32_t* __restrict__ active, int c,
             const double* __restrict__ Vf, double* __restrict__ Vc, double* __restrict__ B,
             const double* __restrict__ KX, const double* __restrict__ KY)
{
    const Where w = locate(L);
    if (w.k < 0 || !active[w.k]) return;
    const KGrid& G = L.g[w.gi];
    const KProb pr = probs[w.k];
    const int64_t cell = (int64_t)w.t * blockDim.x + threadIdx.x;
    const int nx = G.nx, ny = G.ny;
    if (cell >= (int64_t)nx * ny) return;
    const int I = (int)(cell % nx), J = (int)(cell / nx);
    const int fnx = 2 * nx, fny = 2 * ny;
    const double* vf = Vf + pr.arena_base + G.aoff_x;
    const double* bf = B + pr.arena_base + G.aoff_x;
    const double* kx = KX + pr.fx_base + xface_off(c, pr.Qs, G.p + 1, G.q + 1);
    const double* ky = KY + pr.fy_base + yface_off(c, pr.Qs, G.p + 1, G.q + 1);
    const double ihx2 = (double)fnx * fnx, ihy2 = (double)fny * fny;
    const double r00 = residual_at(vf, bf, kx, ky, fnx, fny, 2 * I, 2 * J, ihx2, ihy2);
    const double r10 = residual_at(vf, bf, kx, ky, fnx, fny, 2 * I + 1, 2 * J, ihx2, ihy2);
    const double r01 = residual_at(vf, bf, kx, ky, fnx, fny, 2 * I, 2 * J + 1, ihx2, ihy2);
    const double r11 = residual_at(vf, bf, kx, ky, fnx, fny, 2 * I + 1, 2 * J + 1, ihx2, ihy2);
    B[pr.arena_base + G.aoff + cell] = 0.5 * (0.5 * (r00 + r10) + 0.5 * (r01 + r11));
    Vc[pr.arena_base + G.aoff + cell] = 0.0;
}

// fine grid G += omega * bilinear interpolation (odd reflection at the walls)
// of the coarse iterate of grid (p-1,q-1) at aoff_x
__global__ void __launch_bounds__(kBlock)
k_prolong2d(KLevel L, const KProb* __restrict__ probs, const int32_t* __restrict__ active, double omega,
            const double* __restrict__ Vc, double* __restrict__ Vf)
{
    const Where w = locate(L);
    if (w.k < 0 || !active[w.k]) return;
    const KGrid& G = L.g[w.gi];
    const KProb pr = probs[w.k];
    const int64_t cell = (int64_t)w.t * blockDim.x + threadIdx.x;
    const int nx = G.nx, ny = G.ny;
    if (cell >= (int64_t)nx * ny) return;
    const int i = (int)(cell % nx), j = (int)(cell / nx);
    const int ncx = nx / 2, ncy = ny / 2;
    const double* vc = Vc + pr.arena_base + G.aoff_x;
    const int J = j >> 1, Jn = (j & 1) ? J + 1 : J - 1;
    const double r0 = linear_at(vc + (int64_t)J * ncx, (int64_t)1, ncx, i);
    const double r1 = (Jn >= 0 && Jn < ncy) ? linear_at(vc + (int64_t)Jn * ncx, (int64_t)1, ncx, i) : -r0;
    Vf[pr.arena_base + G.aoff + cell] += omega * (0.75 * r0 + 0.25 * r1);
}

// v = A^-1 b on the coarsest (c x c) grid of each problem, lane k unknown k
__global__ void __launch_bounds__(64)
k_dense_apply(int K, const KProb* __restrict__ probs, const int32_t* __restrict__ active, int n, int64_t aoff,
              const double* __restrict__ inv, double* __restrict__ V, const double* __restrict__ B)
{
    const int k = blockIdx.x;
    if (k >= K || !active[k]) return;
    const KProb pr = probs[k];
    const double* Ai = inv + (int64_t)pr.sample * n * n;
    const double* b = B + pr.arena_base + aoff;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        double x = 0.0;
        for (int j = 0; j < n; ++j) x += Ai[r * n + j] * b[j];
        V[pr.arena_base + aoff + r] = x;
    }
}

// ratio ||b - A v|| / ||b|| of each problem from the residual-norm partial sums
__global__ void __launch_bounds__(64)
k_ratio(int K, int ntiles, const KProb* __restrict__ probs, const double* __restrict__ part,
        double* __restrict__ ratios, int col, int ncols)
{
    const int k = blockIdx.x;
    if (k >= K) return;
    const KProb pr = probs[k];
    double rr = 0.0, bb = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += 64) {
        rr += part[2 * (pr.part_base + t)];
        bb += part[2 * (pr.part_base + t) + 1];
    }
    for (int off = 32; off > 0; off >>= 1) {
        rr += __shfl_down(rr, off, 64);
        bb += __shfl_down(bb, off, 64);
    }
    if (threadIdx.x == 0) ratios[(int64_t)pr.sample * ncols + col] = sqrt(rr) / sqrt(bb);
}

// ------------------------------------------------------------------------
// Quantities of interest of Section 5 per grid, one workgroup per (grid,
// sample): the mean of u; u at (1/2,1/2) by bilinear interpolation of the
// cell centres; the average over [1/4,1/2]^2 of the cell-wise constant
// solution (cells weighted by their overlap); the flux through x = 1, per
// row the wall face's 2 k u / h_x times h_y.  Sums run in a fixed order.
// ------------------------------------------------------------------------
__device__ __forceinline__ double block_sum1(double v)
{
    __shared__ double part[kBlock / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += part[w];
    return t;
}

__global__ void __launch_bounds__(kBlock)
k_qoi(int S, int kind, int c, const int32_t* __restrict__ PQ, const int64_t* __restrict__ cbase,
      const int64_t* __restrict__ xbase, const int64_t* __restrict__ gbase, const double* __restrict__ KX,
      const double* __restrict__ U, double* __restrict__ out)
{
    const int s = blockIdx.y, g = blockIdx.x;
    if (s >= S) return;
    const int P = PQ[2 * s], Qs = PQ[2 * s + 1];
    if (g >= (P + 1) * (Qs + 1)) return;                  // uniform per workgroup
    const int p = g / (Qs + 1), q = g % (Qs + 1);
    const int nx = c << p, ny = c << q;
    const double* u = U + cbase[s] + cell_off(c, Qs, p, q);
    double acc = 0.0;
    if (kind == QOI_MEAN) {
        for (int k = threadIdx.x; k < nx * ny; k += kBlock) acc += u[k];
        acc = block_sum1(acc) / ((double)nx * ny);
    } else if (kind == QOI_POINT) {
        const double tx = 0.5 * nx - 0.5, ty = 0.5 * ny - 0.5;
        const int i0 = (int)floor(tx), j0 = (int)floor(ty);
        const double wx = tx - i0, wy = ty - j0;
        const int i1 = wx > 0.0 ? i0 + 1 : i0, j1 = wy > 0.0 ? j0 + 1 : j0;
        acc = (1.0 - wx) * (1.0 - wy) * u[j0 * nx + i0] + wx * (1.0 - wy) * u[j0 * nx + i1] +
              (1.0 - wx) * wy * u[j1 * nx + i0] + wx * wy * u[j1 * nx + i1];
    } else if (kind == QOI_SUBDOMAIN) {
        // cells overlapping [1/4,1/2] in each direction
        const int ia = (nx / 4), ib = (nx + 1) / 2, ja = (ny / 4), jb = (ny + 1) / 2;
        const int w = ib - ia, h = jb - ja;
        for (int k = threadIdx.x; k < w * h; k += kBlock) {
            const int i = ia + k % w, j = ja + k / w;
            const double ox = fmin((i + 1.0) / nx, 0.5) - fmax((double)i / nx, 0.25);
            const double oy = fmin((j + 1.0) / ny, 0.5) - fmax((double)j / ny, 0.25);
            if (ox > 0.0 && oy > 0.0) acc += u[j * nx + i] * ox * oy;
        }
        acc = block_sum1(acc) / 0.0625;
    } else {
        const double* kx = KX + xbase[s] + xface_off(c, Qs, p, q);
        for (int j = threadIdx.x; j < ny; j += kBlock)
            acc += 2.0 * kx[j * (nx + 1) + nx] * u[j * nx + nx - 1] * (double)nx / (double)ny;
        acc = block_sum1(acc);
    }
    if (threadIdx.x == 0) out[gbase[s] + g] = acc;
}

// ------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------
#define LAUNCH_CHECK() (hipGetLastError())

hipError_t launch_field(const FieldArgs& A, int nsamples, const int32_t* samples, const SampleBase* bases,
                        const double* xi, double* kx, double* ky, float* kx32, float* ky32, hipStream_t st)
{
    const int fw = A.kind_faces == 0 ? A.nx + 1 : A.nx, fh = A.kind_faces == 0 ? A.ny : A.ny + 1;
    const int tiles = ((fw + kFieldTI - 1) / kFieldTI) * ((fh + kFieldTJ - 1) / kFieldTJ);
    const size_t lds = sizeof(double) * ((size_t)A.Mx * A.My + (size_t)A.Mx * kFieldTI + (size_t)A.Mx * kFieldTJ);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_field, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_field, dim3(tiles, nsamples), dim3(kBlock), lds, st, A, samples, bases, xi, kx, ky, kx32, ky32);
    return LAUNCH_CHECK();
}

hipError_t launch_face_mean(int c, int p, int q, int kind_faces, int nsamples, const int32_t* samples,
                            const SampleBase* bases, double* kx, double* ky, float* kx32, float* ky32, hipStream_t st)
{
    const int nx = c << p, ny = c << q;
    const int64_t n = kind_faces == 0 ? (int64_t)(nx + 1) * ny : (int64_t)nx * (ny + 1);
    hipLaunchKernelGGL(k_face_mean, dim3((unsigned)((n + kBlock - 1) / kBlock), nsamples), dim3(kBlock), 0, st, c, p,
                       q, kind_faces, samples, bases, kx, ky, kx32, ky32);
    return LAUNCH_CHECK();
}

hipError_t launch_kl_xi(int S, int n_terms, uint64_t seed, const int64_t* ids, double* xi, hipStream_t st)
{
    const int64_t n = (int64_t)S * ((n_terms + 3) / 4);
    hipLaunchKernelGGL(k_kl_xi, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, S, n_terms, seed, ids,
                       xi);
    return LAUNCH_CHECK();
}

hipError_t launch_chol(int S, int c, const SampleBase* bases, const double* kx, const double* ky, double* chol,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_chol, dim3(S), dim3(64), 2 * sizeof(double) * c * c * c * c, st, S, c, bases, kx, ky, chol);
    return LAUNCH_CHECK();
}

static dim3 level_grid(const KLevel& L, int K) { return dim3((unsigned)(((int64_t)L.ntiles * K + 7) / 8 * 8)); }

static unsigned threads_of(const KLevel& L) { return L.bs > 0 ? (unsigned)L.bs : (unsigned)kBlock; }

static KLevel with_blocks(const KLevel& L, int K)
{
    KLevel c = L;
    c.nblocks = L.ntiles * K;
    return c;
}

template <typename T, int NT>
static void rbgs_dispatch(int ns, bool corr, dim3 grid, size_t lds, hipStream_t st, const KLevel& Lb, const KProb* probs,
                          const int32_t* active, int c, const T* Vin, T* Vout, const T* B, const T* KX, const T* KY,
                          const T* Vc, T omega)
{
    if (ns == 0) {
        hipLaunchKernelGGL((k_rbgs<T, 0, false, NT>), grid, dim3(NT), lds, st, Lb, probs, active, c, Vin, Vout, B, KX, KY, Vc, omega, nullptr, nullptr);
    } else if (corr) {
        if (ns == 1)
            hipLaunchKernelGGL((k_rbgs<T, 1, true, NT>), grid, dim3(NT), lds, st, Lb, probs, active, c, Vin, Vout, B, KX, KY, Vc, omega, nullptr, nullptr);
        else
            hipLaunchKernelGGL((k_rbgs<T, 2, true, NT>), grid, dim3(NT), lds, st, Lb, probs, active, c, Vin, Vout, B, KX, KY, Vc, omega, nullptr, nullptr);
    } else {
        if (ns == 1)
            hipLaunchKernelGGL((k_rbgs<T, 1, false, NT>), grid, dim3(NT), lds, st, Lb, probs, active, c, Vin, Vout, B, KX, KY, Vc, omega, nullptr, nullptr);
        else
            hipLaunchKernelGGL((k_rbgs<T, 2, false, NT>), grid, dim3(NT), lds, st, Lb, probs, active, c, Vin, Vout, B, KX, KY, Vc, omega, nullptr, nullptr);
    }
}

template <typename T>
hipError_t launch_rbgs(int ns, const KLevel& L, int K, const KProb* probs, const int32_t* active, int c,
                       const T* Vin, T* Vout, const T* B, const T* KX, const T* KY, const T* Vc, T omega,
                       hipStream_t st)
{
    const dim3 grid = level_grid(L, K);
    const KLevel Lb = with_blocks(L, K);
    const size_t lds = sizeof(T) * (size_t)L.lds;
    if (L.bs == 64)
        rbgs_dispatch<T, 64>(ns, Vc != nullptr, grid, lds, st, Lb, probs, active, c, Vin, Vout, B, KX, KY, Vc, omega);
    else
        rbgs_dispatch<T, kBlock>(ns, Vc != nullptr, grid, lds, st, Lb, probs, active, c, Vin, Vout, B, KX, KY, Vc,
                                 omega);
    return LAUNCH_CHECK();
}

template <typename T>
hipError_t launch_rbgs_restrict(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c,
                                const T* Vin, T* Vout, T* B, const T* KX, const T* KY, T* Vco, hipStream_t st)
{
    const dim3 grid = level_grid(L, K);
    const KLevel Lb = with_blocks(L, K);
    const size_t lds = sizeof(T) * (size_t)L.lds;
    if (L.bs == 64)
        hipLaunchKernelGGL((k_rbgs<T, 2, false, 64, true>), grid, dim3(64), lds, st, Lb, probs, active, c, Vin, Vout, B,
                           KX, KY, nullptr, T(0), B, Vco);
    else
        hipLaunchKernelGGL((k_rbgs<T, 2, false, kBlock, true>), grid, dim3(kBlock), lds, st, Lb, probs, active, c, Vin,
                           Vout, B, KX, KY, nullptr, T(0), B, Vco);
    return LAUNCH_CHECK();
}

template <typename T>
hipError_t launch_rbgs_corr_restrict(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c,
                                     const T* Vin, T* Vout, T* B, const T* KX, const T* KY, const T* Vc, T omega,
                                     T* Vco, hipStream_t st)
{
    const dim3 grid = level_grid(L, K);
    const KLevel Lb = with_blocks(L, K);
    const size_t lds = sizeof(T) * (size_t)L.lds;
    if (L.bs == 64)
        hipLaunchKernelGGL((k_rbgs<T, 4, true, 64, true>), grid, dim3(64), lds, st, Lb, probs, active, c, Vin, Vout, B,
                           KX, KY, Vc, omega, B, Vco);
    else
        hipLaunchKernelGGL((k_rbgs<T, 4, true, kBlock, true>), grid, dim3(kBlock), lds, st, Lb, probs, active, c, Vin,
                           Vout, B, KX, KY, Vc, omega, B, Vco);
    return LAUNCH_CHECK();
}

template <typename T>
hipError_t launch_rb_colour(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c, int colour,
                            T* V, const T* B, const T* KX, const T* KY, hipStream_t st)
{
    hipLaunchKernelGGL((k_rb_colour<T>), level_grid(L, K), dim3(threads_of(L)), 0, st, with_blocks(L, K), probs,
                       active, c, colour, V, B, KX, KY);
    return LAUNCH_CHECK();
}

template <typename T>
hipError_t launch_restrict_combine(const KLevel& L, int K, const KProb* probs, const int32_t* active, T* Vc, T* B,
                                   hipStream_t st)
{
    hipLaunchKernelGGL((k_restrict_combine<T>), level_grid(L, K), dim3(threads_of(L)), 0, st, with_blocks(L, K), probs,
                       active, Vc, B);
    return LAUNCH_CHECK();
}

template <typename T>
hipError_t launch_restrict(bool rhs, const KLevel& L, int K, const KProb* probs, const int32_t* active, int c,
                           const T* Vf, T* Vc, T* B, const T* KX, const T* KY, hipStream_t st)
{
    if (rhs)
        hipLaunchKernelGGL((k_restrict<T, true>), level_grid(L, K), dim3(threads_of(L)), 0, st, with_blocks(L, K), probs, active, c, Vf, Vc, B, KX, KY);
    else
        hipLaunchKernelGGL((k_restrict<T, false>), level_grid(L, K), dim3(threads_of(L)), 0, st, with_blocks(L, K), probs, active, c, Vf, Vc, B, KX, KY);
    return LAUNCH_CHECK();
}

template <typename T>
hipError_t launch_prolong(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c, T omega,
                          const T* Vc, T* Vf, const T* KX, const T* KY, hipStream_t st)
{
    hipLaunchKernelGGL((k_prolong<T>), level_grid(L, K), dim3(threads_of(L)), 0, st, with_blocks(L, K), probs, active, c, omega, Vc, Vf, KX, KY);
    return LAUNCH_CHECK();
}

template <typename T>
hipError_t launch_tail(const KTail* tables, const int32_t* cls, int tidx, int kbase, int threads, size_t lds_bytes,
                       int K, const KProb* probs, const int32_t* active, int c, int mu, int nu1, int nu2, T omega,
                       int count, int combine, T* V, T* B, const T* KX, const T* KY, const T* pack,
                       const double* chol, const TailSolve& ad, hipStream_t st)
{
    const void* fn = threads == 256 ? (const void*)k_tail<T, 256> : (const void*)k_tail<T, 64>;
    if (lds_bytes > 65536) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return e;
    }
    if (threads == 256)
        hipLaunchKernelGGL((k_tail<T, 256>), dim3(K), dim3(256), lds_bytes, st, tables, cls, tidx, kbase, probs,
                           active, c, mu, nu1, nu2, omega, count, combine, V, B, KX, KY, pack, chol, ad);
    else
        hipLaunchKernelGGL((k_tail<T, 64>), dim3(K), dim3(64), lds_bytes, st, tables, cls, tidx, kbase, probs,
                           active, c, mu, nu1, nu2, omega, count, combine, V, B, KX, KY, pack, chol, ad);
    return LAUNCH_CHECK();
}

hipError_t launch_tail_slots(const KTail* table, int4* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_tail_slots, dim3(1), dim3(kBlock), 0, st, table, out);
    return LAUNCH_CHECK();
}

template <typename T>
hipError_t launch_tail_pack(const KTail* table, int K, const KProb* probs, int c, const T* KX, const T* KY, T* pack,
                            hipStream_t st)
{
    hipLaunchKernelGGL((k_tail_pack<T>), dim3(K), dim3(kBlock), 0, st, table, probs, c, KX, KY, pack);
    return LAUNCH_CHECK();
}

hipError_t launch_fmg(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c, double* V, double* B,
                      const double* U, const double* BP, const double* KX, const double* KY, hipStream_t st)
{
    hipLaunchKernelGGL(k_fmg, level_grid(L, K), dim3(kBlock), 0, st, with_blocks(L, K), probs, active, c, V, B, U, BP, KX, KY);
    return LAUNCH_CHECK();
}

hipError_t launch_resnorm(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c, const double* V,
                          const double* B, const double* KX, const double* KY, double* part, float* V32, float* B32,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_resnorm, level_grid(L, K), dim3(kBlock), 0, st, with_blocks(L, K), probs, active, c, V, B, KX, KY, part, V32, B32);
    return LAUNCH_CHECK();
}

hipError_t launch_converge(int K, int ntiles, const KProb* probs, int32_t* active, int32_t* pcycles,
                           int32_t* dead_level, int32_t* status, const double* part, double tol, int max_cycles,
                           int level, int32_t* n_active, hipStream_t st)
{
    hipLaunchKernelGGL(k_converge, dim3(K), dim3(64), 0, st, K, ntiles, probs, active, pcycles, dead_level, status, part,
                       tol, max_cycles, level, n_active);
    return LAUNCH_CHECK();
}

hipError_t launch_ir_update(const KLevel& L, int K, const KProb* probs, const int32_t* active, double* V,
                            const float* V32, hipStream_t st)
{
    hipLaunchKernelGGL(k_ir_update, level_grid(L, K), dim3(kBlock), 0, st, with_blocks(L, K), probs, active, V, V32);
    return LAUNCH_CHECK();
}

hipError_t launch_snapshot(const KLevel& L, int K, const KProb* probs, const int32_t* dead_level, int level, int c,
                           const double* V, double* U, double* part, hipStream_t st)
{
    hipLaunchKernelGGL(k_snapshot, level_grid(L, K), dim3(kBlock), 0, st, with_blocks(L, K), probs, dead_level, level, c, V, U, part);
    return LAUNCH_CHECK();
}

hipError_t launch_qreduce(int K, int ntiles, int64_t cells, const KProb* probs, const int32_t* pcycles,
                          const int64_t* grid_base, const double* part, double* q_out, int32_t* cycles_out,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_qreduce, dim3(K), dim3(64), 0, st, K, ntiles, cells, probs, pcycles, grid_base, part, q_out,
                       cycles_out);
    return LAUNCH_CHECK();
}

hipError_t launch_rhs_top(const KLevel& L, int K, const KProb* probs, double* BP, const double* rhs,
                          const int64_t* rhs_base, hipStream_t st)
{
    hipLaunchKernelGGL(k_rhs_top, level_grid(L, K), dim3(kBlock), 0, st, with_blocks(L, K), probs, BP, rhs, rhs_base);
    return LAUNCH_CHECK();
}

hipError_t launch_activate(int K, const KProb* probs, const int32_t* dead_level, int level, int32_t* active,
                           int32_t* pcycles, hipStream_t st)
{
    hipLaunchKernelGGL(k_activate, dim3((K + kBlock - 1) / kBlock), dim3(kBlock), 0, st, K, probs, dead_level, level,
                       active, pcycles);
    return LAUNCH_CHECK();
}

hipError_t launch_delta_q(int S, int max_grids, const int32_t* PQ, const int64_t* gbase, const double* q, double* dq,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_delta_q, dim3((max_grids + kBlock - 1) / kBlock, S), dim3(kBlock), 0, st, S, PQ, gbase, q, dq);
    return LAUNCH_CHECK();
}

hipError_t launch_plain_init(const KLevel& L, int K, const KProb* probs, const double* rhs, double* V, double* B,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_plain_init, level_grid(L, K), dim3(threads_of(L)), 0, st, with_blocks(L, K), probs, rhs, V, B);
    return LAUNCH_CHECK();
}

hipError_t launch_restrict2d(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c,
                             const double* Vf, double* Vc, double* B, const double* KX, const double* KY,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_restrict2d, level_grid(L, K), dim3(threads_of(L)), 0, st, with_blocks(L, K), probs, active, c,
                       Vf, Vc, B, KX, KY);
    return LAUNCH_CHECK();
}

hipError_t launch_prolong2d(const KLevel& L, int K, const KProb* probs, const int32_t* active, double omega,
                            const double* Vc, double* Vf, hipStream_t st)
{
    hipLaunchKernelGGL(k_prolong2d, level_grid(L, K), dim3(threads_of(L)), 0, st, with_blocks(L, K), probs, active,
                       omega, Vc, Vf);
    return LAUNCH_CHECK();
}

hipError_t launch_dense_apply(int K, const KProb* probs, const int32_t* active, int n, int64_t aoff,
                              const double* inv, double* V, const double* B, hipStream_t st)
{
    hipLaunchKernelGGL(k_dense_apply, dim3(K), dim3(64), 0, st, K, probs, active, n, aoff, inv, V, B);
    return LAUNCH_CHECK();
}

hipError_t launch_ratio(int K, int ntiles, const KProb* probs, const double* part, double* ratios, int col, int ncols,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_ratio, dim3(K), dim3(64), 0, st, K, ntiles, probs, part, ratios, col, ncols);
    return LAUNCH_CHECK();
}

hipError_t launch_qoi(int S, int max_grids, int kind, int c, const int32_t* PQ, const int64_t* cbase,
                      const int64_t* xbase, const int64_t* gbase, const double* KX, const double* U, double* out,
                      hipStream_t st)
{
    hipLaunchKernelGGL(k_qoi, dim3(max_grids, S), dim3(kBlock), 0, st, S, kind, c, PQ, cbase, xbase, gbase, KX, U,
                       out);
    return LAUNCH_CHECK();
}

template hipError_t launch_rbgs<double>(int, const KLevel&, int, const KProb*, const int32_t*, int, const double*,
                                        double*, const double*, const double*, const double*, const double*, double,
                                        hipStream_t);
template hipError_t launch_rbgs<float>(int, const KLevel&, int, const KProb*, const int32_t*, int, const float*,
                                       float*, const float*, const float*, const float*, const float*, float,
                                       hipStream_t);
template hipError_t launch_rbgs_restrict<double>(const KLevel&, int, const KProb*, const int32_t*, int, const double*,
                                                double*, double*, const double*, const double*, double*, hipStream_t);
template hipError_t launch_rbgs_restrict<float>(const KLevel&, int, const KProb*, const int32_t*, int, const float*,
                                               float*, float*, const float*, const float*, float*, hipStream_t);
template hipError_t launch_rbgs_corr_restrict<double>(const KLevel&, int, const KProb*, const int32_t*, int,
                                                      const double*, double*, double*, const double*, const double*,
                                                      const double*, double, double*, hipStream_t);
template hipError_t launch_rbgs_corr_restrict<float>(const KLevel&, int, const KProb*, const int32_t*, int,
                                                     const float*, float*, float*, const float*, const float*,
                                                     const float*, float, float*, hipStream_t);
template hipError_t launch_rb_colour<double>(const KLevel&, int, const KProb*, const int32_t*, int, int, double*,
                                             const double*, const double*, const double*, hipStream_t);
template hipError_t launch_rb_colour<float>(const KLevel&, int, const KProb*, const int32_t*, int, int, float*,
                                            const float*, const float*, const float*, hipStream_t);
template hipError_t launch_restrict_combine<double>(const KLevel&, int, const KProb*, const int32_t*, double*, double*,
                                                    hipStream_t);
template hipError_t launch_restrict_combine<float>(const KLevel&, int, const KProb*, const int32_t*, float*, float*,
                                                   hipStream_t);
template hipError_t launch_restrict<double>(bool, const KLevel&, int, const KProb*, const int32_t*, int,
                                            const double*, double*, double*, const double*, const double*,
                                            hipStream_t);
template hipError_t launch_restrict<float>(bool, const KLevel&, int, const KProb*, const int32_t*, int, const float*,
                                           float*, float*, const float*, const float*, hipStream_t);
template hipError_t launch_prolong<double>(const KLevel&, int, const KProb*, const int32_t*, int, double,
                                           const double*, double*, const double*, const double*, hipStream_t);
template hipError_t launch_prolong<float>(const KLevel&, int, const KProb*, const int32_t*, int, float, const float*,
                                          float*, const float*, const float*, hipStream_t);
template hipError_t launch_tail<double>(const KTail*, const int32_t*, int, int, int, size_t, int, const KProb*,
                                        const int32_t*, int, int, int, int, double, int, int, double*, double*,
                                        const double*, const double*, const double*, const double*,
                                        const TailSolve&, hipStream_t);
template hipError_t launch_tail<float>(const KTail*, const int32_t*, int, int, int, size_t, int, const KProb*,
                                       const int32_t*, int, int, int, int, float, int, int, float*, float*, const float*,
                                       const float*, const float*, const double*, const TailSolve&, hipStream_t);
template hipError_t launch_tail_pack<double>(const KTail*, int, const KProb*, int, const double*, const double*,
                                             double*, hipStream_t);
template hipError_t launch_tail_pack<float>(const KTail*, int, const KProb*, int, const float*, const float*, float*,
                                            hipStream_t);

}  // namespace msg
