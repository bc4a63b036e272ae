// matern_kernels.hpp -- launchers of the circulant-embedding Matern field
// kernels (matern.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msg {

// per-sample parameters of one chunk (device table)
struct MaternSample {
    double t00, t01, t10, t11;   // T = S R
    int64_t id;                  // Philox counter word 1
    int64_t fx_base, fy_base;    // sample's first x- and y-face in the batch arrays
};

hipError_t launch_mat_twiddles(int n_max, double2* tw, hipStream_t st);
hipError_t launch_mat_row(int K, int Mx, int My, double hx, double hy, double nu, double coef,
                          const MaternSample* smp, double2* A, hipStream_t st);
hipError_t launch_fft_rows(int64_t rows, int logn, int tw_stride, const double2* tw, double2* X, hipStream_t st);
hipError_t launch_transpose(int K, int R, int C, const double2* in, double2* out, hipStream_t st);
// FFTs of rows of 2^logn points as 2^h1 x 2^(logn-h1) (four-step; both
// factors at most one workgroup's row length); S: scratch of the same size
hipError_t launch_fft_rows_long(int64_t rows, int logn, int h1, int tw_log, const double2* tw, double2* X,
                                double2* S, hipStream_t st);
hipError_t launch_eig_ratio(int K, int64_t M, int nb, const double2* L, double2* part, const int32_t* out_index,
                            double* ratio, hipStream_t st);
hipError_t launch_mat_xi(int K, int Mx, int My, uint64_t seed, uint64_t key1, const MaternSample* smp, double2* LT,
                         hipStream_t st);
hipError_t launch_mat_faces(int K, int c, int P, int Q, int Mx, int My, const MaternSample* smp, const double2* Y,
                            double* kx, double* ky, float* kx32, float* ky32, hipStream_t st);

}  // namespace msg
