// Surrogate step kernels: the sampled-column judge and the application of
// the plain tendencies of the sampled columns.
//
// Judge (a reading; the paper has no learned component): at step t column c
// is sampled when SplitMix64(seed ^ (t << 32) ^ c) mod rate == 0.  The plain
// physics of the sampled columns is the reference; per variable the RMSE of
// the surrogate's tendencies pooled over the sampled columns and all levels is
// compared with rel * sigma_v (sigma_v: training-set std of that tendency).
// Strictly greater for theta or q means the whole step falls back to the
// plain physics.  Also reported: the fraction of sampled columns whose own
// RMSE (over the levels of one variable) exceeds the same bound.  Sampled columns always take the plain result.  The decision
// stays on the device: later launches read the flag and exit early.
#include "wx_internal.h"
#include "wx_mlp_internal.h"

namespace wx {
namespace {

// ---- deterministic compaction of the sampled column ids -------------------
__global__ void k_sample_count(int ncol, uint64_t seed, uint64_t t, unsigned rate, int *block_count) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  const bool s = c < ncol && judge_sampled(seed, t, unsigned(c), rate);
  const int n = __syncthreads_count(s);
  if (threadIdx.x == 0) block_count[blockIdx.x] = n;
}

// Exclusive scan of the block counts (one block); total into *n_out.  Each
// thread sums a run of counts (loads eight at a time), the 256 run sums are
// scanned in LDS by doubling steps, and each thread writes its run's offsets.
__global__ void k_sample_scan(const int *block_count, int nb, int *block_off, int *n_out) {
  __shared__ int part[256];
  const int t = threadIdx.x;
  const int per = (nb + 255) / 256;
  const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
  int s = 0, b = b0;
  for (; b + 8 <= b1; b += 8) {
    int v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = block_count[b + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; b < b1; ++b) s += block_count[b];
  part[t] = s;
  __syncthreads();
  for (int w = 1; w < 256; w <<= 1) {
    const int v = t >= w ? part[t - w] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  if (t == 255) *n_out = part[255];
  int run = part[t] - s;
  for (b = b0; b + 8 <= b1; b += 8) {
    int v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = block_count[b + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      block_off[b + u] = run;
      run += v[u];
    }
  }
  for (; b < b1; ++b) {
    block_off[b] = run;
    run += block_count[b];
  }
}

// Slot of each sampled column: its block's offset plus the sampled columns
// before it in the block (a ballot within the wavefront, the earlier
// wavefronts' counts from LDS), so the list is in column order.
__global__ void k_sample_write(int ncol, uint64_t seed, uint64_t t, unsigned rate, const int *block_off, int cap,
                               int *list) {
  __shared__ int wcount[4];
  const int c = blockIdx.x * 256 + threadIdx.x;
  const bool s = c < ncol && judge_sampled(seed, t, unsigned(c), rate);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const unsigned long long m = __ballot(s);
  if (lane == 0) wcount[w] = __popcll(m);
  __syncthreads();
  if (s) {
    int before = __popcll(m & ((1ull << lane) - 1ull));
    for (int q = 0; q < w; ++q) before += wcount[q];
    const int slot = block_off[blockIdx.x] + before;
    if (slot < cap) list[slot] = c;
  }
}

// ---- RMSE of the surrogate on the sampled columns, fallback decision -------
// y_hat: normalised outputs [cap][128]; t_ref: plain tendencies [cap][128].
// Two levels in a fixed order: block b sums the squared errors of the
// elements e = b * 256 + t + i * (JUDGE_BLOCKS * 256) (tree within the
// block), then one thread adds the block partials in block order.
constexpr int JUDGE_BLOCKS = 120;
// block partials: 2 doubles per block, then two int counters (see k_judge_cols)
constexpr int JUDGE_COUNT_OFF = 2 * JUDGE_BLOCKS;

__global__ void k_judge_part(const float *y_hat, const float *t_ref, const int *n_list, int cap, const float *ymean,
                             const float *ystd, int nz, double *part) {
  __shared__ double sh[2][256];
  const int t = threadIdx.x;
  const int n = min(*n_list, cap);
  const long long total = (long long)n * TEND_ROW;
  double e[2] = {0.0, 0.0};
  // elements x = first, first + stride, ... summed in that order; their loads
  // go out eight at a time (a loop with one load pair per element waits a
  // memory round trip per element)
  constexpr long long stride = (long long)JUDGE_BLOCKS * 256;
  auto add = [&](long long x, float yh, float tr) {
    const int o = int(x % TEND_ROW);
    if (o >= 2 * nz) return;
    const double pred = double(yh) * ystd[o] + ymean[o];
    const double d = pred - double(tr);
    e[o >= nz] += d * d;
  };
  long long x = (long long)blockIdx.x * 256 + t;
  for (; x + 7 * stride < total; x += 8 * stride) {
    float yh[8], tr[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      yh[u] = y_hat[x + u * stride];
      tr[u] = t_ref[x + u * stride];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) add(x + u * stride, yh[u], tr[u]);
  }
  for (; x < total; x += stride) add(x, y_hat[x], t_ref[x]);
  sh[0][t] = e[0];
  sh[1][t] = e[1];
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) {
      sh[0][t] += sh[0][t + w];
      sh[1][t] += sh[1][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[2 * blockIdx.x] = sh[0][0];
    part[2 * blockIdx.x + 1] = sh[1][0];
    if (blockIdx.x == 0) {
      int *cnt = reinterpret_cast<int *>(part + JUDGE_COUNT_OFF);
      cnt[0] = 0;
      cnt[1] = 0;
    }
  }
}

// Per sampled column: its own RMSE over the levels of each variable against
// the same bound; counts the columns that exceed it (integer atomics, so the
// counts do not depend on the order).
__global__ void k_judge_cols(const float *y_hat, const float *t_ref, const int *n_list, int cap, const float *ymean,
                             const float *ystd, const double *sigma, double rel, int nz, double *part) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= min(*n_list, cap)) return;
  double e[2] = {0.0, 0.0};
  // outputs in order, their loads eight at a time
  const float *yr = y_hat + (size_t)s * TEND_ROW, *tr = t_ref + (size_t)s * TEND_ROW;
  int o = 0;
  for (; o + 8 <= 2 * nz; o += 8) {
    float a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a[u] = yr[o + u];
      b[u] = tr[o + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double d = (double(a[u]) * ystd[o + u] + ymean[o + u]) - double(b[u]);
      e[o + u >= nz] += d * d;
    }
  }
  for (; o < 2 * nz; ++o) {
    const double pred = double(yr[o]) * ystd[o] + ymean[o];
    const double d = pred - double(tr[o]);
    e[o >= nz] += d * d;
  }
  int *cnt = reinterpret_cast<int *>(part + JUDGE_COUNT_OFF);
  for (int v = 0; v < 2; ++v)
    if (sqrt(e[v] / nz) > rel * sigma[v]) atomicAdd(&cnt[v], 1);
}

__global__ void k_judge_final(const double *part, const int *n_list, int cap, const double *sigma, double rel, int nz,
                              int *fallback, double *judge_out, int *flags) {
  if (threadIdx.x != 0) return;
  const int n = min(*n_list, cap);
  double e0 = 0.0, e1 = 0.0;
  for (int b = 0; b < JUDGE_BLOCKS; ++b) {
    e0 += part[2 * b];
    e1 += part[2 * b + 1];
  }
  const double cnt = double(n) * nz;
  const double r0 = n > 0 ? sqrt(e0 / cnt) : 0.0;
  const double r1 = n > 0 ? sqrt(e1 / cnt) : 0.0;
  const int fb = (r0 > rel * sigma[0]) || (r1 > rel * sigma[1]);
  *fallback = fb;
  const int *over = reinterpret_cast<const int *>(part + JUDGE_COUNT_OFF);
  judge_out[0] = r0;
  judge_out[1] = r1;
  judge_out[2] = fb;
  judge_out[3] = n;
  judge_out[4] = n > 0 ? double(over[0]) / n : 0.0;
  judge_out[5] = n > 0 ? double(over[1]) / n : 0.0;
  if (fb) atomicAdd(&flags[3], 1);
}

// ---- apply the plain tendencies of the sampled columns ---------------------
// Plain tendencies of the sampled columns (rows by slot), unless falling back.
template <typename T>
__global__ void k_apply_sampled(ApplyArgs<T> a, const float *tend, const int *list, const int *n_list, int cap) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= min(*n_list, cap)) return;
  if (a.fallback && *a.fallback) return;
  const int c = list[s];
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int i = c % nx, j = c / nx;
  const unsigned g0 = a.g.origin + unsigned(i) + unsigned(j) * a.g.sj;
  const int di = i < 2 ? nx : (i >= nx - 2 ? -nx : 0);
  const int dj = j < 2 ? ny * int(a.g.sj) : (j >= ny - 2 ? -ny * int(a.g.sj) : 0);
  const float *row = tend + (size_t)s * TEND_ROW;
  if (a.tend_t) {
    for (int k = 0; k < nz; ++k) {
      const unsigned o = unsigned(k * ny + j) * unsigned(nx) + unsigned(i);
      stg(a.tend_t, o, row[k]);
      stg(a.tend_q, o, row[nz + k]);
    }
    return;
  }
  for (int k = 0; k < nz; ++k) {
    const unsigned g = g0 + unsigned(k) * a.g.sk;
    const T tn = ldg(a.th, g) + a.dt * T(row[k]);
    const T qn = ldg(a.q, g) + a.dt * T(row[nz + k]);
    stg(a.th, g, tn);
    stg(a.q, g, qn);
    if (di != 0) { stg(a.th, g + di, tn); stg(a.q, g + di, qn); }
    if (dj != 0) {
      stg(a.th, g + dj, tn); stg(a.q, g + dj, qn);
      if (di != 0) { stg(a.th, g + dj + di, tn); stg(a.q, g + dj + di, qn); }
    }
  }
}

}  // namespace

hipError_t launch_sample(int ncol, uint64_t seed, uint64_t t, unsigned rate, int *block_count, int *block_off,
                         int *n_list, int cap, int *list, hipStream_t s) {
  const int nb = (ncol + 255) / 256;
  hipLaunchKernelGGL(k_sample_count, dim3(nb), dim3(256), 0, s, ncol, seed, t, rate, block_count);
  hipLaunchKernelGGL(k_sample_scan, dim3(1), dim3(256), 0, s, block_count, nb, block_off, n_list);
  hipLaunchKernelGGL(k_sample_write, dim3(nb), dim3(256), 0, s, ncol, seed, t, rate, block_off, cap, list);
  return hipGetLastError();
}

hipError_t launch_judge(const float *y_hat, const float *t_ref, const int *n_list, int cap, const float *ymean,
                        const float *ystd, const double *sigma, double rel, int nz, double *part, int *fallback,
                        double *judge_out, int *flags, hipStream_t s) {
  hipLaunchKernelGGL(k_judge_part, dim3(JUDGE_BLOCKS), dim3(256), 0, s, y_hat, t_ref, n_list, cap, ymean, ystd, nz,
                     part);
  if (cap > 0)
    hipLaunchKernelGGL(k_judge_cols, dim3((cap + 127) / 128), dim3(128), 0, s, y_hat, t_ref, n_list, cap, ymean, ystd,
                       sigma, rel, nz, part);
  hipLaunchKernelGGL(k_judge_final, dim3(1), dim3(64), 0, s, part, n_list, cap, sigma, rel, nz, fallback, judge_out,
                     flags);
  return hipGetLastError();
}

size_t judge_part_bytes() { return size_t(2) * JUDGE_BLOCKS * sizeof(double) + 2 * sizeof(int); }

template <typename T>
hipError_t launch_apply_sampled(const ApplyArgs<T> &a, const float *tend, const int *list, const int *n_list, int cap,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_apply_sampled<T>, dim3((cap + 127) / 128), dim3(128), 0, s, a, tend, list, n_list, cap);
  return hipGetLastError();
}

template hipError_t launch_apply_sampled<float>(const ApplyArgs<float> &, const float *, const int *, const int *, int,
                                                hipStream_t);
template hipError_t launch_apply_sampled<double>(const ApplyArgs<double> &, const float *, const int *, const int *,
                                                 int, hipStream_t);

}  // namespace wx
