// C ABI of the learned surrogate (include/wx.h): parameter-blob layout,
// initialisation, normalisation, training step, inference.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "wx.h"
#include "wx_internal.h"
#include "wx_mlp_internal.h"

namespace wx {
int set_error(int code, const char *msg);
}

namespace {

using namespace wx;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return wx::set_error(code, buf);
}

#define MLP_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) return fail(WX_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// element counts of the six parameter tensors (padded shapes)
const size_t kParamElems[6] = {size_t(MLP_NHID) * MLP_KIN, MLP_NHID, size_t(MLP_NHID) * MLP_NHID, MLP_NHID,
                               size_t(MLP_NOUTP) * MLP_NHID, MLP_NOUTP};

size_t section_bytes(int s) {
  if (s < 24) return kParamElems[s % 6] * 4;
  switch (s) {
    case WX_MLP_W1_BF16: return kParamElems[0] * 2;
    case WX_MLP_W2_BF16: return kParamElems[2] * 2;
    case WX_MLP_W3_BF16: return kParamElems[4] * 2;
    case WX_MLP_W2T_BF16: return kParamElems[2] * 2;
    case WX_MLP_W3T_BF16: return kParamElems[4] * 2;
    case WX_MLP_X_MEAN: case WX_MLP_X_INVSTD: return MLP_KIN * 4;
    case WX_MLP_Y_MEAN: case WX_MLP_Y_STD: return MLP_NOUTP * 4;
    case WX_MLP_SIGMA: return 2 * 4;
    case WX_MLP_SIGMA64: return 2 * 8;
    case WX_MLP_WPACK_BF16: return (kParamElems[0] + kParamElems[2] + kParamElems[4]) * 2;
  }
  return 0;
}

size_t section_offset(int s) {
  size_t off = 0;
  for (int q = 0; q < s; ++q) off += a256(section_bytes(q));
  return off;
}

template <typename T>
T *sec(void *blob, int s) {
  return reinterpret_cast<T *>(static_cast<unsigned char *>(blob) + section_offset(s));
}
template <typename T>
const T *sec(const void *blob, int s) {
  return reinterpret_cast<const T *>(static_cast<const unsigned char *>(blob) + section_offset(s));
}

// Fragment-order copy of weight matrix l (0: W1, 1: W2, 2: W3) in the blob.
uint16_t *packed_weights(void *blob, int l) {
  size_t off = 0;
  if (l > 0) off += kParamElems[0];
  if (l > 1) off += kParamElems[2];
  return sec<uint16_t>(blob, WX_MLP_WPACK_BF16) + off;
}

bool al16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Training workspace for a batch of B rows.
struct Work {
  uint16_t *h1, *h2, *d3b, *g2b, *g1b;
  float *y, *d3f, *g2f, *g1f, *row_loss;
  float *part3, *part2, *part1;            // split-K slices of dW3, dW2, dW1
  float *cp2, *cp1;                        // 32-row column sums of the hidden gradients
  size_t total;
  static constexpr int kSplitRows = 256;   // batch rows per dW split
};

Work work_layout(void *base, int B) {
  Work w{};
  unsigned char *p = static_cast<unsigned char *>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char *r = p ? p + off : nullptr;
    off += a256(bytes);
    return r;
  };
  w.h1 = reinterpret_cast<uint16_t *>(take(size_t(B) * MLP_NHID * 2));
  w.h2 = reinterpret_cast<uint16_t *>(take(size_t(B) * MLP_NHID * 2));
  w.d3b = reinterpret_cast<uint16_t *>(take(size_t(B) * MLP_NOUTP * 2));
  w.g2b = reinterpret_cast<uint16_t *>(take(size_t(B) * MLP_NHID * 2));
  w.g1b = reinterpret_cast<uint16_t *>(take(size_t(B) * MLP_NHID * 2));
  w.y = reinterpret_cast<float *>(take(size_t(B) * MLP_NOUTP * 4));
  w.d3f = reinterpret_cast<float *>(take(size_t(B) * MLP_NOUTP * 4));
  w.g2f = reinterpret_cast<float *>(take(size_t(B) * MLP_NHID * 4));
  w.g1f = reinterpret_cast<float *>(take(size_t(B) * MLP_NHID * 4));
  w.row_loss = reinterpret_cast<float *>(take(size_t(B) * 4));
  const size_t splits = (size_t(B) + Work::kSplitRows - 1) / Work::kSplitRows;
  w.part3 = reinterpret_cast<float *>(take(splits * MLP_NOUTP * MLP_NHID * 4));
  w.part2 = reinterpret_cast<float *>(take(splits * MLP_NHID * MLP_NHID * 4));
  w.part1 = reinterpret_cast<float *>(take(splits * MLP_NHID * MLP_KIN * 4));
  w.cp2 = reinterpret_cast<float *>(take(size_t((B + 31) / 32) * MLP_NHID * 4));
  w.cp1 = reinterpret_cast<float *>(take(size_t((B + 31) / 32) * MLP_NHID * 4));
  w.total = off;
  return w;
}

// The three layers for rows x[rows[m]] (or x[m] when rows is null), m < n.
int forward_layers(const void *blob, const uint16_t *x, const int *rows, int n, uint16_t *h1, uint16_t *h2, float *y,
                   hipStream_t st) {
  GemmSpec g{};
  g.a_kcontig = g.b_kcontig = true;
  g.splits = 1;
  g.M = n;
  // layer 1 (gathering the batch rows on the way into LDS)
  g.A = x; g.lda = MLP_KIN; g.rows_a = rows; g.B = sec<uint16_t>(blob, WX_MLP_W1_BF16); g.ldb = MLP_KIN;
  g.N = MLP_NHID; g.K = MLP_KIN; g.bias = sec<float>(blob, WX_MLP_B1); g.C = h1; g.ldc = MLP_NHID;
  g.epilogue = GEMM_BIAS_RELU_BF16;
  MLP_HIP(launch_gemm(g, st));
  g.rows_a = nullptr;
  // layer 2
  g.A = h1; g.lda = MLP_NHID; g.B = sec<uint16_t>(blob, WX_MLP_W2_BF16); g.ldb = MLP_NHID;
  g.N = MLP_NHID; g.K = MLP_NHID; g.bias = sec<float>(blob, WX_MLP_B2); g.C = h2; g.ldc = MLP_NHID;
  MLP_HIP(launch_gemm(g, st));
  // layer 3
  g.A = h2; g.lda = MLP_NHID; g.B = sec<uint16_t>(blob, WX_MLP_W3_BF16); g.ldb = MLP_NHID;
  g.N = MLP_NOUTP; g.K = MLP_NHID; g.bias = sec<float>(blob, WX_MLP_B3); g.C = y; g.ldc = MLP_NOUTP;
  g.epilogue = GEMM_BIAS_F32;
  MLP_HIP(launch_gemm(g, st));
  return WX_OK;
}

// dW[n][k] = sum_m d[m][n] act[act_rows[m]][k] over the batch (act row m when
// act_rows is null) as split-K partial slices; *job describes their ordered
// sum into out (run by launch_grad_finish).
GemmSpec weight_grad(const uint16_t *d, int ldd, int nout, const uint16_t *act, const int *act_rows, int lda, int kin,
                     int B, float *part, float *out, SplitJob *job, int split_rows = Work::kSplitRows) {
  GemmSpec g{};
  g.a_kcontig = g.b_kcontig = false;
  g.A = d; g.lda = ldd; g.B = act; g.ldb = lda; g.rows_b = act_rows;
  g.M = nout; g.N = kin; g.K = B;
  g.splits = (B + split_rows - 1) / split_rows;
  g.C = part; g.ldc = kin; g.split_stride = size_t(nout) * kin;
  g.epilogue = GEMM_PARTIAL_F32;
  const int k_split = ((B + g.splits - 1) / g.splits + 31) / 32 * 32;
  const int nsplit = (B + k_split - 1) / k_split;
  const int n = nout * kin;
  *job = {part, nsplit, g.split_stride, out, n, (n + 255) / 256};
  return g;
}

// Hidden-layer gradient: g = (sum_n d[m][n] W[n][k]) * (h[m][k] > 0), with W
// given transposed as [k][n]; FP32 into out and its BF16 operand into out16.
GemmSpec input_grad(const uint16_t *d, int ldd, int nred, const uint16_t *wt, int kout, int B, const uint16_t *h,
                    float *out, uint16_t *out16, float *colpart) {
  GemmSpec g{};
  g.a_kcontig = g.b_kcontig = true;
  g.A = d; g.lda = ldd; g.B = wt; g.ldb = nred;
  g.M = B; g.N = kout; g.K = nred; g.splits = 1;
  g.C = out; g.ldc = kout; g.epilogue = GEMM_MASK_F32_BF16;
  g.mask = h; g.C2 = out16; g.colpart = colpart;
  return g;
}

// Adam step t with rate lr over the six parameter tensors of the blob (their
// gradients, moments and BF16 copies).
AdamArgs adam_args(void *blob, float lr, int t) {
  uint16_t *wb[6] = {sec<uint16_t>(blob, WX_MLP_W1_BF16), nullptr, sec<uint16_t>(blob, WX_MLP_W2_BF16), nullptr,
                     sec<uint16_t>(blob, WX_MLP_W3_BF16), nullptr};
  uint16_t *wbt[6] = {nullptr, nullptr, sec<uint16_t>(blob, WX_MLP_W2T_BF16), nullptr,
                      sec<uint16_t>(blob, WX_MLP_W3T_BF16), nullptr};
  uint16_t *wbp[6] = {packed_weights(blob, 0), nullptr, packed_weights(blob, 1), nullptr, packed_weights(blob, 2),
                      nullptr};
  const int rows[6] = {MLP_NHID, 1, MLP_NHID, 1, MLP_NOUTP, 1};
  const int cols[6] = {MLP_KIN, MLP_NHID, MLP_NHID, MLP_NHID, MLP_NHID, MLP_NOUTP};
  AdamArgs aa{};
  aa.lr = lr;
  aa.bc1 = float(1.0 - std::pow(0.9, t));
  aa.bc2 = float(1.0 - std::pow(0.999, t));
  size_t start = 0;
  for (int p = 0; p < 6; ++p) {
    aa.seg[p] = {sec<float>(blob, p), sec<float>(blob, WX_MLP_GRAD + p), sec<float>(blob, WX_MLP_ADAM_M + p),
                 sec<float>(blob, WX_MLP_ADAM_V + p), wb[p], wbt[p], wbp[p], start, kParamElems[p], rows[p], cols[p]};
    start += kParamElems[p];
  }
  return aa;
}

// Forward, loss and backward for one batch; with adam non-null the finishing
// launch also applies the Adam step to every parameter as its gradient forms.
int forward_backward(void *blob, void *work, const void *x, const float *y, const int32_t *rows, int batch,
                     float *loss_sum, const AdamArgs *adam, void *stream) {
  if (!blob || !work || !x || !y || !rows || !loss_sum) return fail(WX_E_INVAL, "NULL argument");
  if (batch < 1 || batch > 65536) return fail(WX_E_INVAL, "batch must be in 1..65536");
  if (!al16(blob) || !al16(work) || !al16(x)) return fail(WX_E_INVAL, "blob, work and x must be 16-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Work w = work_layout(work, batch);
  const int B = batch;
  const uint16_t *xs = static_cast<const uint16_t *>(x);
  if (int rc = forward_layers(blob, xs, rows, B, w.h1, w.h2, w.y, st)) return rc;
  MLP_HIP(launch_loss(w.y, y, rows, B, MLP_NOUT, MLP_NOUTP, w.d3f, w.d3b, w.row_loss, st));
  GradFinishArgs gf{};
  gf.nsj = 3;
  // output layer and hidden layer 2 in one launch: both read the output
  // delta (the ReLU mask and BF16 rounding of the hidden gradient in its
  // GEMM's epilogue)
  MLP_HIP(launch_gemm_pair(weight_grad(w.d3b, MLP_NOUTP, MLP_NOUTP, w.h2, nullptr, MLP_NHID, MLP_NHID, B, w.part3,
                                       sec<float>(blob, WX_MLP_GRAD + 4), &gf.sj[0]),
                           input_grad(w.d3b, MLP_NOUTP, MLP_NOUTP, sec<uint16_t>(blob, WX_MLP_W3T_BF16), MLP_NHID, B,
                                      w.h2, w.g2f, w.g2b, w.cp2),
                           st));
  // hidden layer 2's weights and hidden layer 1: both read its delta
  MLP_HIP(launch_gemm_pair(weight_grad(w.g2b, MLP_NHID, MLP_NHID, w.h1, nullptr, MLP_NHID, MLP_NHID, B, w.part2,
                                       sec<float>(blob, WX_MLP_GRAD + 2), &gf.sj[1], 2 * Work::kSplitRows),
                           input_grad(w.g2b, MLP_NHID, MLP_NHID, sec<uint16_t>(blob, WX_MLP_W2T_BF16), MLP_NHID, B,
                                      w.h1, w.g1f, w.g1b, w.cp1),
                           st));
  MLP_HIP(launch_gemm(weight_grad(w.g1b, MLP_NHID, MLP_NHID, xs, rows, MLP_KIN, MLP_KIN, B, w.part1,
                                  sec<float>(blob, WX_MLP_GRAD + 0), &gf.sj[2]),
                      st));
  // one launch for the rest, fixed order: the weight gradients (ordered sums
  // of their split-K slices), the bias gradients (column sums of the
  // unrounded FP32 deltas) and the loss (sum of the per-row sums)
  ColsumArgs &cs = gf.cs;
  cs.rows = B;
  cs.njobs = 4;
  cs.job[0] = {w.d3f, MLP_NOUTP, MLP_NOUTP, sec<float>(blob, WX_MLP_GRAD + 5), MLP_NOUTP / COLSUM_COLS, 1};
  // (the hidden layers' bias gradients from their GEMMs' 32-row column sums)
  cs.job[1] = {w.cp2, MLP_NHID, MLP_NHID, sec<float>(blob, WX_MLP_GRAD + 3), MLP_NHID / COLSUM_COLS, 1, (B + 31) / 32};
  cs.job[2] = {w.cp1, MLP_NHID, MLP_NHID, sec<float>(blob, WX_MLP_GRAD + 1), MLP_NHID / COLSUM_COLS, 1, (B + 31) / 32};
  cs.job[3] = {w.row_loss, 1, 1, loss_sum, 1, 0};
  if (adam) {
    gf.adam = *adam;
    gf.adam_on = 1;
    gf.sj_seg[0] = 4; gf.sj_seg[1] = 2; gf.sj_seg[2] = 0;                    // dW3, dW2, dW1
    gf.cs_seg[0] = 5; gf.cs_seg[1] = 3; gf.cs_seg[2] = 1; gf.cs_seg[3] = -1;  // db3, db2, db1, loss
  }
  MLP_HIP(launch_grad_finish(gf, st));
  return WX_OK;
}

}  // namespace

extern "C" {

size_t wx_mlp_bytes(void) { return section_offset(WX_MLP_NSECTIONS); }

int64_t wx_mlp_offset(int section) {
  if (section < 0 || section >= WX_MLP_NSECTIONS) return -1;
  return int64_t(section_offset(section));
}

int wx_mlp_refresh(void *blob, void *stream) {
  if (!blob || !al16(blob)) return fail(WX_E_INVAL, "blob is NULL or misaligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  MLP_HIP(launch_to_bf16(sec<float>(blob, WX_MLP_W1), kParamElems[0], sec<uint16_t>(blob, WX_MLP_W1_BF16), nullptr,
                         packed_weights(blob, 0), MLP_NHID, MLP_KIN, st));
  MLP_HIP(launch_to_bf16(sec<float>(blob, WX_MLP_W2), kParamElems[2], sec<uint16_t>(blob, WX_MLP_W2_BF16),
                         sec<uint16_t>(blob, WX_MLP_W2T_BF16), packed_weights(blob, 1), MLP_NHID, MLP_NHID, st));
  MLP_HIP(launch_to_bf16(sec<float>(blob, WX_MLP_W3), kParamElems[4], sec<uint16_t>(blob, WX_MLP_W3_BF16),
                         sec<uint16_t>(blob, WX_MLP_W3T_BF16), packed_weights(blob, 2), MLP_NOUTP, MLP_NHID, st));
  return WX_OK;
}

int wx_mlp_init(void *blob, uint64_t seed, void *stream) {
  if (!blob || !al16(blob)) return fail(WX_E_INVAL, "blob is NULL or misaligned");
  if (seed >= (1ull << 32)) return fail(WX_E_INVAL, "seed must be < 2^32");
  hipStream_t st = static_cast<hipStream_t>(stream);
  // zero everything (a fill kernel), then draw the weights into their real
  // (unpadded) blocks
  MLP_HIP(launch_fill_i32(static_cast<int *>(blob), int(wx_mlp_bytes() / 4), 0, st));
  const int fan_out[3] = {MLP_NHID, MLP_NHID, MLP_NOUT};
  const int fan_in[3] = {MLP_NIN, MLP_NHID, MLP_NHID};
  const int ld[3] = {MLP_KIN, MLP_NHID, MLP_NHID};
  for (int l = 0; l < 3; ++l) {
    const float bound = float(std::sqrt(6.0 / fan_in[l]));
    MLP_HIP(launch_he_init(sec<float>(blob, 2 * l), ld[l], fan_out[l], fan_in[l], seed, 2 * l, bound, st));
  }
  // identity normalisation: mean 0, 1/std 1 on real features, std 1
  std::vector<float> ones(MLP_KIN, 1.f);
  for (int f = MLP_NIN; f < MLP_KIN; ++f) ones[f] = 0.f;
  MLP_HIP(hipMemcpyAsync(sec<float>(blob, WX_MLP_X_INVSTD), ones.data(), MLP_KIN * 4, hipMemcpyHostToDevice, st));
  std::vector<float> ys(MLP_NOUTP, 1.f);
  MLP_HIP(hipMemcpyAsync(sec<float>(blob, WX_MLP_Y_STD), ys.data(), MLP_NOUTP * 4, hipMemcpyHostToDevice, st));
  MLP_HIP(hipStreamSynchronize(st));   // the host vectors above go out of scope
  return wx_mlp_refresh(blob, stream);
}

size_t wx_mlp_norm_scratch_bytes(size_t n) { return fit_norm_scratch_bytes(n); }

int wx_mlp_fit_norm(void *blob, const float *x_raw, const float *y_raw, size_t n, void *scratch, void *stream) {
  if (!blob || !x_raw || !y_raw || !scratch || n == 0) return fail(WX_E_INVAL, "NULL argument or n == 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  MLP_HIP(launch_fit_norm(x_raw, y_raw, n, static_cast<double *>(scratch), sec<float>(blob, WX_MLP_X_MEAN),
                          sec<float>(blob, WX_MLP_X_INVSTD), sec<float>(blob, WX_MLP_Y_MEAN),
                          sec<float>(blob, WX_MLP_Y_STD), sec<float>(blob, WX_MLP_SIGMA),
                          sec<double>(blob, WX_MLP_SIGMA64), st));
  return WX_OK;
}

int wx_mlp_normalize(const void *blob, const float *x_raw, const float *y_raw, size_t n, void *x_out, float *y_out,
                     void *stream) {
  if (!blob || !x_raw || !x_out || (y_raw && !y_out)) return fail(WX_E_INVAL, "NULL argument");
  if (!al16(x_out)) return fail(WX_E_INVAL, "x_out must be 16-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  MLP_HIP(launch_normalize(x_raw, y_raw, n, sec<float>(blob, WX_MLP_X_MEAN), sec<float>(blob, WX_MLP_X_INVSTD),
                           sec<float>(blob, WX_MLP_Y_MEAN), sec<float>(blob, WX_MLP_Y_STD),
                           static_cast<uint16_t *>(x_out), y_out, st));
  return WX_OK;
}

size_t wx_mlp_work_bytes(int batch) {
  if (batch < 1 || batch > 65536) return 0;
  return work_layout(nullptr, batch).total;
}

int wx_mlp_forward_backward(void *blob, void *work, const void *x, const float *y, const int32_t *rows, int batch,
                            float *loss_sum, void *stream) {
  return forward_backward(blob, work, x, y, rows, batch, loss_sum, nullptr, stream);
}

int wx_mlp_adam(void *blob, float lr, int t, void *stream) {
  if (!blob || !al16(blob)) return fail(WX_E_INVAL, "blob is NULL or misaligned");
  if (t < 1 || !(lr >= 0.f)) return fail(WX_E_INVAL, "t must be >= 1 and lr >= 0");
  MLP_HIP(launch_adam_multi(adam_args(blob, lr, t), static_cast<hipStream_t>(stream)));
  return WX_OK;
}

int wx_mlp_train_step(void *blob, void *work, const void *x, const float *y, const int32_t *rows, int batch, float lr,
                      int t, float *loss_sum, void *stream) {
  if (!blob || !al16(blob)) return fail(WX_E_INVAL, "blob is NULL or misaligned");
  if (t < 1 || !(lr >= 0.f)) return fail(WX_E_INVAL, "t must be >= 1 and lr >= 0");
  // the Adam step runs inside the launch that forms the gradients
  const AdamArgs aa = adam_args(blob, lr, t);
  return forward_backward(blob, work, x, y, rows, batch, loss_sum, &aa, stream);
}

int wx_mlp_shuffle(uint64_t seed, uint64_t epoch, int n, int m, int32_t *out, void *stream) {
  if (n < 0 || n > (1 << 30) || m < 0 || m > n) return fail(WX_E_INVAL, "need 0 <= m <= n <= 2^30");
  if (m > 0 && !out) return fail(WX_E_INVAL, "out is NULL");
  MLP_HIP(launch_shuffle(seed, epoch, n, m, out, static_cast<hipStream_t>(stream)));
  return WX_OK;
}

size_t wx_mlp_infer_work_bytes(int n) {
  if (n < 1) return 0;
  return 2 * a256(size_t(n) * MLP_NHID * 2);
}

int wx_mlp_infer(const void *blob, void *work, const void *x, int n, float *y_out, void *stream) {
  if (!blob || !work || !x || !y_out || n < 1) return fail(WX_E_INVAL, "NULL argument or n < 1");
  if (!al16(blob) || !al16(work) || !al16(x)) return fail(WX_E_INVAL, "blob, work and x must be 16-byte aligned");
  uint16_t *h1 = static_cast<uint16_t *>(work);
  uint16_t *h2 = reinterpret_cast<uint16_t *>(static_cast<unsigned char *>(work) + a256(size_t(n) * MLP_NHID * 2));
  return forward_layers(blob, static_cast<const uint16_t *>(x), nullptr, n, h1, h2, y_out, static_cast<hipStream_t>(stream));
}

}  // extern "C"
