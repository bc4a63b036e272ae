// msg_kernels.hpp -- launch wrappers of the HIP kernels (msg_kernels.hip),
// called by the host scheduler (msg_host.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msg_device.hpp"

namespace msg {

enum { MSG_ST_CONVERGED = 0, MSG_ST_MAXITER = 1, MSG_ST_NONFINITE = 2 };

// where a sample's arrays start, and its rectangle
struct SampleBase {
    int64_t fx, fy;        // first x-face / y-face
    int32_t P, Q;
};

// adaptive cycling inside the tail kernel (count < 0)
struct TailSolve {
    double tol;
    int32_t max_cycles;
    int32_t level;
    int32_t* pcycles;      // per problem, offset like the problem table
    int32_t* status;       // per sample
    int32_t* dead_level;   // per sample
};

// one launch of the field synthesis: one face kind of one grid (p,q) for a
// list of samples sharing that grid
struct FieldArgs {
    int32_t kind;          // 0: cosine table, 1: separable squared-exponential
    int32_t n_terms;       // xi values per sample
    int32_t Mx, My;        // coefficient matrix C[Mx][My] of cos(pi m x) cos(pi n y)
    int32_t c, p, q, nx, ny;
    int32_t kind_faces;    // 0: x-faces, 1: y-faces
    double sigma;
    double lamx[kMaxModes], lamy[kMaxModes];
    KCosTable cos;
};

hipError_t launch_field(const FieldArgs& A, int nsamples, const int32_t* samples, const SampleBase* bases,
                        const double* xi, double* kx, double* ky, float* kx32, float* ky32, hipStream_t st);
// the faces of grid (p,q) (kind 0: x, 1: y) of each listed sample as means of
// its finest grid's faces (MSG_FACE_MEAN); the finest grids must be filled
hipError_t launch_face_mean(int c, int p, int q, int kind_faces, int nsamples, const int32_t* samples,
                            const SampleBase* bases, double* kx, double* ky, float* kx32, float* ky32, hipStream_t st);
// standard normals xi[S][n_terms] of the streams (seed, ids[s])
hipError_t launch_kl_xi(int S, int n_terms, uint64_t seed, const int64_t* ids, double* xi, hipStream_t st);
hipError_t launch_chol(int S, int c, const SampleBase* bases, const double* kx, const double* ky, double* chol,
                       hipStream_t st);
// Vc != nullptr: the pass first adds omega * (coarse-grid correction from the
// grids at L.g[].aoff_x / aoff_y of Vc) to the iterate (eq. interpolation)
template <typename T>
hipError_t launch_rbgs(int ns, const KLevel& L, int K, const KProb* probs, const int32_t* active, int c,
                       const T* Vin, T* Vout, const T* B, const T* KX, const T* KY, const T* Vc, T omega,
                       hipStream_t st);
// a two-sweep pass that also restricts its residual into level l-1, and the
// combination of the two halves on coarse grids with two parents
template <typename T>
hipError_t launch_rbgs_restrict(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c,
                                const T* Vin, T* Vout, T* B, const T* KX, const T* KY, T* Vco, hipStream_t st);
template <typename T>
hipError_t launch_restrict_combine(const KLevel& L, int K, const KProb* probs, const int32_t* active, T* Vc, T* B,
                                   hipStream_t st);
// the post-smoothing pass of one W-cycle visit (correction from Vc, two
// sweeps) and the restricting pre-smoothing pass of the next visit (two
// sweeps, residual restricted into Vco and B) as one pass
template <typename T>
hipError_t launch_rbgs_corr_restrict(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c,
                                     const T* Vin, T* Vout, T* B, const T* KX, const T* KY, const T* Vc, T omega,
                                     T* Vco, hipStream_t st);
// one colour of a red-black half-sweep in place in global memory (L: one
// thread per cell; the split-sweep debug mode)
template <typename T>
hipError_t launch_rb_colour(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c, int colour,
                            T* V, const T* B, const T* KX, const T* KY, hipStream_t st);
template <typename T>
hipError_t launch_restrict(bool rhs, const KLevel& L, int K, const KProb* probs, const int32_t* active, int c,
                           const T* Vf, T* Vc, T* B, const T* KX, const T* KY, hipStream_t st);
template <typename T>
hipError_t launch_prolong(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c, T omega,
                          const T* Vc, T* Vf, const T* KX, const T* KY, hipStream_t st);
// block b uses class descriptor tables[cls[b]] (cls given, -1 skips the
// block) or tables[tidx] and is problem kbase + b of the stage (which picks
// its conductance image in `pack`); threads is 64 or 256; combine != 0 when the top
// level was just filled by the restricting pre-smoothing pass, whose two
// halves of a grid with two parents the tail averages as it loads them
hipError_t launch_tail_slots(const KTail* table, int4* out, hipStream_t st);
template <typename T>
hipError_t launch_tail(const KTail* tables, const int32_t* cls, int tidx, int kbase, int threads, size_t lds_bytes,
                       int K,
                       const KProb* probs, const int32_t* active, int c, int mu, int nu1, int nu2, T omega,
                       int count, int combine, T* V, T* B, const T* KX, const T* KY, const T* pack,
                       const double* chol, const TailSolve& ad, hipStream_t st);
// the conductance image of the tail of each of K problems (pack: K * nstat elements)
template <typename T>
hipError_t launch_tail_pack(const KTail* table, int K, const KProb* probs, int c, const T* KX, const T* KY, T* pack,
                            hipStream_t st);
hipError_t launch_fmg(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c, double* V, double* B,
                      const double* U, const double* BP, const double* KX, const double* KY, hipStream_t st);
hipError_t launch_resnorm(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c, const double* V,
                          const double* B, const double* KX, const double* KY, double* part, float* V32, float* B32,
                          hipStream_t st);
hipError_t launch_converge(int K, int ntiles, const KProb* probs, int32_t* active, int32_t* pcycles,
                           int32_t* dead_level, int32_t* status, const double* part, double tol, int max_cycles,
                           int level, int32_t* n_active, hipStream_t st);
hipError_t launch_ir_update(const KLevel& L, int K, const KProb* probs, const int32_t* active, double* V,
                            const float* V32, hipStream_t st);
hipError_t launch_snapshot(const KLevel& L, int K, const KProb* probs, const int32_t* dead_level, int level, int c,
                           const double* V, double* U, double* part, hipStream_t st);
hipError_t launch_qreduce(int K, int ntiles, int64_t cells, const KProb* probs, const int32_t* pcycles,
                          const int64_t* grid_base, const double* part, double* q_out, int32_t* cycles_out,
                          hipStream_t st);
hipError_t launch_rhs_top(const KLevel& L, int K, const KProb* probs, double* BP, const double* rhs,
                          const int64_t* rhs_base, hipStream_t st);
// plain cycles from zero and standard multigrid (one grid per level, full coarsening)
hipError_t launch_plain_init(const KLevel& L, int K, const KProb* probs, const double* rhs, double* V, double* B,
                             hipStream_t st);
hipError_t launch_restrict2d(const KLevel& L, int K, const KProb* probs, const int32_t* active, int c,
                             const double* Vf, double* Vc, double* B, const double* KX, const double* KY,
                             hipStream_t st);
hipError_t launch_prolong2d(const KLevel& L, int K, const KProb* probs, const int32_t* active, double omega,
                            const double* Vc, double* Vf, hipStream_t st);
hipError_t launch_dense_apply(int K, const KProb* probs, const int32_t* active, int n, int64_t aoff,
                              const double* inv, double* V, const double* B, hipStream_t st);
hipError_t launch_ratio(int K, int ntiles, const KProb* probs, const double* part, double* ratios, int col, int ncols,
                        hipStream_t st);
// quantities of interest (the same values as the C-ABI's MSG_QOI_*)
enum QoiKind { QOI_MEAN = 0, QOI_POINT = 1, QOI_SUBDOMAIN = 2, QOI_FLUX = 3 };
// quantity of interest `kind` of every grid of S samples
hipError_t launch_qoi(int S, int max_grids, int kind, int c, const int32_t* PQ, const int64_t* cbase,
                      const int64_t* xbase, const int64_t* gbase, const double* KX, const double* U, double* out,
                      hipStream_t st);
hipError_t launch_delta_q(int S, int max_grids, const int32_t* PQ, const int64_t* gbase, const double* q, double* dq,
                          hipStream_t st);
hipError_t launch_activate(int K, const KProb* probs, const int32_t* dead_level, int level, int32_t* active,
                           int32_t* pcycles, hipStream_t st);

}  // namespace msg
