// Internal interface of the surrogate kernels (k_mlp.hip, k_surrogate.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "wx_internal.h"

namespace wx {

constexpr int MLP_NZ = 58;
constexpr int MLP_NIN = 5 * MLP_NZ + 4;    // 294 inputs
constexpr int MLP_KIN = 320;               // padded input width
constexpr int MLP_NHID = 512;
constexpr int MLP_NOUT = 2 * MLP_NZ;       // 116 outputs
constexpr int MLP_NOUTP = 128;             // padded output width

enum GemmEpilogue { GEMM_F32 = 0, GEMM_BIAS_F32 = 1, GEMM_BIAS_RELU_BF16 = 2, GEMM_PARTIAL_F32 = 3 };

// C[m][n] = sum_k A(m,k) B(k,n).  a_kcontig: A is [M][lda] (k contiguous),
// else [K][lda] (m contiguous); likewise B as [N][ldb] or [K][ldb].
struct GemmSpec {
  const uint16_t *A, *B;
  int lda, ldb;
  bool a_kcontig, b_kcontig;
  int M, N, K;
  int splits;                  // > 1: split K, write partial slices
  const int *rows_a;           // optional gather of A rows (a_kcontig only)
  const float *bias;
  void *C;
  int ldc;
  size_t split_stride;
  int epilogue;
};

hipError_t launch_gemm(const GemmSpec &g, hipStream_t s);
hipError_t launch_sum_splits(const float *part, int nsplit, size_t stride, float *out, size_t n, hipStream_t s);
hipError_t launch_loss(const float *y, const float *t, const int *rows, int batch, int nout, int ldy, float *d32,
                       uint16_t *d16, float *row_loss, hipStream_t s);
hipError_t launch_colsum(const float *a, int rows, int cols, int lda, float *part, float *out, hipStream_t s);
hipError_t launch_mask_round(float *a, const uint16_t *mask, size_t n, uint16_t *out, hipStream_t s);
hipError_t launch_adam(float *w, const float *g, float *m, float *v, size_t n, float lr, float bc1, float bc2,
                       uint16_t *wb, uint16_t *wbt, int rows, int cols, hipStream_t s);
hipError_t launch_to_bf16(const float *w, size_t n, uint16_t *wb, uint16_t *wbt, int rows, int cols, hipStream_t s);
hipError_t launch_he_init(float *w, int ld, int fan_out, int fan_in, uint64_t seed, int tensor, float bound,
                          hipStream_t s);

}  // namespace wx

namespace wx {

template <typename T>
struct FeatArgs {
  const T *rho, *th, *q, *u, *v;
  const T *th_s, *q_s, *f0, *ch;
  Geom g;
  double theta_off;
  int mode;                    // 0: raw FP32 rows, 1: normalised BF16 rows
  float *out_f32;
  uint16_t *out_bf16;
  const float *mean, *inv_std; // mode 1
  // rows: row r is column c0 + r (r < nrows), or list[r] when list is set
  // (rows at or beyond *n_list are written as zeros)
  int c0, nrows;
  const int *list, *n_list;
};

template <typename T>
struct ApplyArgs {
  T *th, *q;
  Geom g;
  T dt;
  const float *ymean, *ystd;   // de-normalisation of the surrogate rows
  const int *fallback;         // skip everything when *fallback != 0 (may be null)
  int judged;                  // skip sampled columns
  uint64_t seed, t;
  unsigned rate;
};

template <typename T>
hipError_t launch_features(const FeatArgs<T> &a, hipStream_t s);
hipError_t launch_fit_norm(const float *xr, const float *yr, size_t n, double *scratch, float *xm, float *xis,
                           float *ym, float *ys, float *sig, double *sig64, hipStream_t s);
size_t fit_norm_scratch_bytes(size_t n);
hipError_t launch_normalize(const float *xr, const float *yr, size_t n, const float *xm, const float *xis,
                            const float *ym, const float *ys, uint16_t *xo, float *yo, hipStream_t s);
hipError_t launch_gather_rows(const uint16_t *x, const int *rows, int batch, uint16_t *out, hipStream_t s);

hipError_t launch_sample(int ncol, uint64_t seed, uint64_t t, unsigned rate, int *block_count, int *block_off,
                         int *n_list, int cap, int *list, hipStream_t s);
hipError_t launch_judge(const float *y_hat, const float *t_ref, const int *n_list, int cap, const float *ymean,
                        const float *ystd, const double *sigma, double rel, int nz, int *fallback, double *judge_out,
                        int *flags, hipStream_t s);
template <typename T>
hipError_t launch_apply_surrogate(const ApplyArgs<T> &a, const float *y, int c0, int n, hipStream_t s);
template <typename T>
hipError_t launch_apply_sampled(const ApplyArgs<T> &a, const float *tend, const int *list, const int *n_list, int cap,
                                hipStream_t s);

}  // namespace wx
