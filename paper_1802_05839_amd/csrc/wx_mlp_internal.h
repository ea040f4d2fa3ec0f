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

// FP32 -> BF16 bits, round to nearest even, on the conversion instruction of
// the target (v_cvt_pk_bf16_f32; NaN stays NaN); f2bf2 packs two values, the
// first in the low half.
typedef float wx_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 wx_bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f2bf2(float lo, float hi) {
  const wx_f32x2 v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, wx_bf16x2));
}
__device__ __forceinline__ uint16_t f2bf(float x) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(x)); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// Position of element (r, c) of a [N][K] BF16 matrix in matrix-core fragment
// order: block (r / 32, c / 16) is 512 contiguous values, lane
// r % 32 + 32 ((c % 16) / 8) holding its 8 consecutive k values.
__host__ __device__ __forceinline__ size_t frag_index(int r, int c, int K) {
  const size_t blk = size_t(r >> 5) * size_t(K >> 4) + size_t(c >> 4);
  return (blk * 64 + size_t((r & 31) + 32 * ((c & 15) >> 3))) * 8 + size_t(c & 7);
}

// SplitMix64 output for state increment x (Steele, Lea & Flood 2014).
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Judge sampling: column c is checked against the plain physics at step t.
__device__ __forceinline__ bool judge_sampled(uint64_t seed, uint64_t t, unsigned c, unsigned rate) {
  return splitmix64(seed ^ (t << 32) ^ uint64_t(c)) % rate == 0;
}

// Column values of one level entering the features: theta - 300 K, q and the
// cell-centred winds (FP32).
struct LevelVals {
  float th, q, u, v;
};

// Returns x as a rounded FP32 register value: the optimiser cannot fuse the
// operation that produced x into the one that consumes it (a product into the
// normalisation's subtraction, say), so every kernel rounds alike.
__device__ __forceinline__ float settle(float x) {
  asm volatile("" : "+v"(x));
  return x;
}

// The five feature values of level k from the values of levels k and k - 1:
// theta and q (k = 0) or their differences, the wind speed (k = 0) or the
// shear S = |(u, v)_k - (u, v)_{k-1}|, and S times the two differences.  Both
// feature kernels call this, so their rows agree bit for bit.
__device__ __forceinline__ void level_features(int k, const LevelVals &c, const LevelVals &b, float out[5]) {
  if (k == 0) {
    out[0] = c.th;
    out[1] = c.q;
    out[2] = settle(sqrtf(fmaf(c.u, c.u, settle(c.v * c.v))));
    out[3] = 0.f;
    out[4] = 0.f;
  } else {
    const float dth = settle(c.th - b.th), dq = settle(c.q - b.q);
    const float du = settle(c.u - b.u), dv = settle(c.v - b.v);
    const float sh = settle(sqrtf(fmaf(du, du, settle(dv * dv))));
    out[0] = dth;
    out[1] = dq;
    out[2] = sh;
    out[3] = settle(sh * dth);
    out[4] = settle(sh * dq);
  }
}

enum GemmEpilogue { GEMM_F32 = 0, GEMM_BIAS_F32 = 1, GEMM_BIAS_RELU_BF16 = 2, GEMM_PARTIAL_F32 = 3,
                   GEMM_MASK_F32_BF16 = 4 };

// C[m][n] = sum_k A(m,k) B(k,n).  a_kcontig: A is [M][lda] (k contiguous),
// else [K][lda] (m contiguous); likewise B as [N][ldb] or [K][ldb].
struct GemmSpec {
  const uint16_t *A, *B;
  int lda, ldb;
  bool a_kcontig, b_kcontig;
  int M, N, K;
  int splits;                  // > 1: split K, write partial slices
  const int *rows_a;           // optional gather of A rows (a_kcontig only)
  const int *rows_b;           // optional gather of B's k rows (!b_kcontig only)
  const float *bias;
  void *C;
  int ldc;
  size_t split_stride;
  int epilogue;
  // GEMM_MASK_F32_BF16: C (FP32) and C2 (BF16) = acc where mask (BF16, same
  // layout as C) is > 0, else 0; with colpart set also colpart[m / 32][n] =
  // the sum of C over rows m / 32 * 32 .. + 31 (a fixed order)
  const uint16_t *mask;
  uint16_t *C2;
  float *colpart;
};

hipError_t launch_gemm(const GemmSpec &g, hipStream_t s);
// A weight-gradient GEMM (GEMM_PARTIAL_F32) and an independent hidden-layer
// gradient GEMM (GEMM_MASK_F32_BF16) in one launch; each output is bit for bit
// that of its own launch_gemm.
hipError_t launch_gemm_pair(const GemmSpec &weight_grad, const GemmSpec &input_grad, hipStream_t s);
hipError_t launch_loss(const float *y, const float *t, const int *rows, int batch, int nout, int ldy, float *d32,
                       uint16_t *d16, float *row_loss, hipStream_t s);

// Adam over the six parameter tensors in one launch.
struct AdamSeg {
  float *w;
  const float *g;
  float *m, *v;
  uint16_t *wb, *wbt;   // BF16 copy and transpose (may be null)
  uint16_t *wbp;        // BF16 copy in fragment order (may be null)
  size_t start, n;      // range in the concatenation
  int rows, cols;
};
struct AdamArgs {
  AdamSeg seg[6];
  float lr, bc1, bc2;
};
// Column sums of up to four matrices (fixed order), run inside launch_grad_finish.
constexpr int COLSUM_COLS = 16;  // columns per column-sum block
struct ColsumJob {
  const float *a;   // [rows][lda]; rows = ColsumArgs::rows unless this job's rows > 0
  int cols, lda;
  float *out;       // [cols]
  int blocks;       // (cols + COLSUM_COLS - 1) / COLSUM_COLS
  int vec;          // cols and lda multiples of 4, a 16-byte aligned
  int rows;         // > 0: this job's row count
};
struct ColsumArgs {
  ColsumJob job[4];
  int njobs, rows;
};

// The end of the backward pass in one launch: the column sums of ColsumArgs,
// then the weight gradients as ordered sums of their split-K partial slices.
struct SplitJob {
  const float *part;   // [nsplit][stride]
  int nsplit;
  size_t stride;
  float *out;          // [n], n <= stride
  int n, blocks;       // blocks = (n + 255) / 256
};
struct GradFinishArgs {
  SplitJob sj[3];
  int nsj;
  ColsumArgs cs;
  // optional Adam step on each gradient element as it is formed: split job j
  // updates tensor adam.seg[sj_seg[j]], column-sum job j tensor
  // adam.seg[cs_seg[j]] (-1: no update, the loss)
  AdamArgs adam;
  int adam_on;
  int sj_seg[3], cs_seg[4];
};
hipError_t launch_grad_finish(const GradFinishArgs &a, hipStream_t s);
hipError_t launch_shuffle(uint64_t seed, uint64_t epoch, int n, int m, int32_t *out, hipStream_t s);

hipError_t launch_adam_multi(const AdamArgs &a, hipStream_t s);
hipError_t launch_to_bf16(const float *w, size_t n, uint16_t *wb, uint16_t *wbt, uint16_t *wbp, int rows, int cols,
                          hipStream_t s);
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
  const float *ymean, *ystd;   // unused by the sampled-column apply
  const int *fallback;         // skip everything when *fallback != 0 (may be null)
  int judged;                  // skip sampled columns
  uint64_t seed, t;
  unsigned rate;
  float *tend_t, *tend_q;      // when set: write the rows as flat tendencies, state untouched
};

template <typename T>
hipError_t launch_features(const FeatArgs<T> &a, hipStream_t s);
hipError_t launch_fit_norm(const float *xr, const float *yr, size_t n, double *scratch, float *xm, float *xis,
                           float *ym, float *ys, float *sig, double *sig64, hipStream_t s);
size_t fit_norm_scratch_bytes(size_t n);
hipError_t launch_normalize(const float *xr, const float *yr, size_t n, const float *xm, const float *xis,
                            const float *ym, const float *ys, uint16_t *xo, float *yo, hipStream_t s);

hipError_t launch_sample(int ncol, uint64_t seed, uint64_t t, unsigned rate, int *block_count, int *block_off,
                         int *n_list, int cap, int *list, hipStream_t s);
hipError_t launch_judge(const float *y_hat, const float *t_ref, const int *n_list, int cap, const float *ymean,
                        const float *ystd, const double *sigma, double rel, int nz, double *part, int *fallback,
                        double *judge_out, int *flags, hipStream_t s);
size_t judge_part_bytes();     // FP64 block partials of launch_judge
template <typename T>
hipError_t launch_apply_sampled(const ApplyArgs<T> &a, const float *tend, const int *list, const int *n_list, int cap,
                                hipStream_t s);

// Fused surrogate physics on an FP32 state: feature rows, the three network
// layers and either the tendency update of the state (apply mode) or the
// normalised output rows of listed columns (rows mode), in one launch.
struct FusedArgs {
  const float *rho, *u, *v;
  float *th, *q;                   // feature inputs; updated in apply mode
  const float *th_s, *q_s, *f0, *ch;
  Geom g;
  double theta_off;
  const uint16_t *w1, *w2, *w3;    // BF16 [512][320], [512][512], [128][512], fragment order
  const float *b1, *b2, *b3;
  const float *xmean, *xinvstd, *ymean, *ystd;
  float dt;
  // apply mode (rows_out == null): columns c0 + r for r < ncols
  int c0, ncols;
  const int *fallback;             // nothing happens when *fallback != 0 (may be null)
  int judged;                      // leave the judge's sampled columns alone
  uint64_t seed, t;
  unsigned rate;
  // rows mode: row s < min(*n_list, cap) (s < cap when n_list is null) is
  // column list[s], or column s when list is null; normalised outputs to
  // rows_out[s][128]; an index outside the grid gives the row of zero features
  const int *list, *n_list;
  int cap;
  float *rows_out;
  // tendency mode (apply mode with tend_t set): the de-normalised tendencies
  // go to tend_t / tend_q (nx*ny*nz, i fastest) and the state is not touched
  float *tend_t, *tend_q;
};

hipError_t launch_surrogate_fused(const FusedArgs &a, hipStream_t s);

}  // namespace wx
