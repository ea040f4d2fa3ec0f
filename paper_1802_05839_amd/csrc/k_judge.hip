// Surrogate step kernels: the sampled-column judge and the application of
// predicted tendencies.
//
// Judge (a reading; the paper has no learned component): at step t column c
// is sampled when SplitMix64(seed ^ (t << 32) ^ c) mod rate == 0.  The plain
// physics of the sampled columns is the reference; per variable the RMSE of
// the surrogate's tendencies pooled over the sampled columns and all levels is
// compared with rel * sigma_v (sigma_v: training-set std of that tendency).
// Strictly greater for theta or q means the whole step falls back to the
// plain physics.  Sampled columns always take the plain result.  The decision
// stays on the device: later launches read the flag and exit early.
#include "wx_internal.h"
#include "wx_mlp_internal.h"

namespace wx {
namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ bool sampled(uint64_t seed, uint64_t t, unsigned c, unsigned rate) {
  return splitmix64(seed ^ (t << 32) ^ uint64_t(c)) % rate == 0;
}

// ---- deterministic compaction of the sampled column ids -------------------
__global__ void k_sample_count(int ncol, uint64_t seed, uint64_t t, unsigned rate, int *block_count) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  const bool s = c < ncol && sampled(seed, t, unsigned(c), rate);
  const int n = __syncthreads_count(s);
  if (threadIdx.x == 0) block_count[blockIdx.x] = n;
}

// Exclusive scan of the block counts (one block); total into *n_out.
__global__ void k_sample_scan(const int *block_count, int nb, int *block_off, int *n_out) {
  __shared__ int part[256];
  const int t = threadIdx.x;
  const int per = (nb + 255) / 256;
  const int b0 = t * per, b1 = min(nb, b0 + per);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += block_count[b];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int q = 0; q < 256; ++q) {
      const int v = part[q];
      part[q] = run;
      run += v;
    }
    *n_out = run;
  }
  __syncthreads();
  int run = part[t];
  for (int b = b0; b < b1; ++b) {
    block_off[b] = run;
    run += block_count[b];
  }
}

__global__ void k_sample_write(int ncol, uint64_t seed, uint64_t t, unsigned rate, const int *block_off, int cap,
                               int *list) {
  __shared__ int flags[256];
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int s = (c < ncol && sampled(seed, t, unsigned(c), rate)) ? 1 : 0;
  flags[threadIdx.x] = s;
  __syncthreads();
  if (s) {
    int before = 0;
    for (int q = 0; q < threadIdx.x; ++q) before += flags[q];
    const int slot = block_off[blockIdx.x] + before;
    if (slot < cap) list[slot] = c;
  }
}

// ---- RMSE of the surrogate on the sampled columns, fallback decision -------
// y_hat: normalised outputs [cap][128]; t_ref: plain tendencies [cap][128].
__global__ void k_judge(const float *y_hat, const float *t_ref, const int *n_list, int cap, const float *ymean,
                        const float *ystd, const double *sigma, double rel, int nz, int *fallback,
                        double *judge_out, int *flags) {
  __shared__ double sh[2][256];
  const int t = threadIdx.x;
  const int n = min(*n_list, cap);
  double e[2] = {0.0, 0.0};
  for (int s = t; s < n; s += 256)
    for (int v = 0; v < 2; ++v)
      for (int k = 0; k < nz; ++k) {
        const int o = v * nz + k;
        const double pred = double(y_hat[(size_t)s * TEND_ROW + o]) * ystd[o] + ymean[o];
        const double d = pred - double(t_ref[(size_t)s * TEND_ROW + o]);
        e[v] += d * d;
      }
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
    const double cnt = double(n) * nz;
    const double r0 = n > 0 ? sqrt(sh[0][0] / cnt) : 0.0;
    const double r1 = n > 0 ? sqrt(sh[1][0] / cnt) : 0.0;
    const int fb = (r0 > rel * sigma[0]) || (r1 > rel * sigma[1]);
    *fallback = fb;
    judge_out[0] = r0;
    judge_out[1] = r1;
    judge_out[2] = fb;
    judge_out[3] = n;
    if (fb) atomicAdd(&flags[3], 1);
  }
}

// ---- apply tendencies ---------------------------------------------------------
// Surrogate rows (normalised) for columns [c0, c0 + n): theta += dt T_theta,
// q += dt T_q, with the periodic halo images; skipped entirely when the
// fallback flag is set, and per column when the column is sampled (judged).
template <typename T>
__global__ void k_apply_surrogate(ApplyArgs<T> a, const float *y, int c0, int n) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  if (a.fallback && *a.fallback) return;
  const int c = c0 + r;
  if (a.judged && sampled(a.seed, a.t, unsigned(c), a.rate)) return;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int i = c % nx, j = c / nx;
  const unsigned g0 = a.g.origin + unsigned(i) + unsigned(j) * a.g.sj;
  const int di = i < 2 ? nx : (i >= nx - 2 ? -nx : 0);
  const int dj = j < 2 ? ny * int(a.g.sj) : (j >= ny - 2 ? -ny * int(a.g.sj) : 0);
  const float *row = y + (size_t)r * TEND_ROW;
  for (int k = 0; k < nz; ++k) {
    const unsigned g = g0 + unsigned(k) * a.g.sk;
    const T tn = ldg(a.th, g) + a.dt * T(row[k] * a.ystd[k] + a.ymean[k]);
    const T qn = ldg(a.q, g) + a.dt * T(row[nz + k] * a.ystd[nz + k] + a.ymean[nz + k]);
    stg(a.th, g, tn);
    stg(a.q, g, qn);
    if (di != 0) { stg(a.th, g + di, tn); stg(a.q, g + di, qn); }
    if (dj != 0) {
      stg(a.th, g + dj, tn); stg(a.q, g + dj, qn);
      if (di != 0) { stg(a.th, g + dj + di, tn); stg(a.q, g + dj + di, qn); }
    }
  }
}

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
                        const float *ystd, const double *sigma, double rel, int nz, int *fallback, double *judge_out,
                        int *flags, hipStream_t s) {
  hipLaunchKernelGGL(k_judge, dim3(1), dim3(256), 0, s, y_hat, t_ref, n_list, cap, ymean, ystd, sigma, rel, nz,
                     fallback, judge_out, flags);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_surrogate(const ApplyArgs<T> &a, const float *y, int c0, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_surrogate<T>, dim3((n + 127) / 128), dim3(128), 0, s, a, y, c0, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_sampled(const ApplyArgs<T> &a, const float *tend, const int *list, const int *n_list, int cap,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_apply_sampled<T>, dim3((cap + 127) / 128), dim3(128), 0, s, a, tend, list, n_list, cap);
  return hipGetLastError();
}

template hipError_t launch_apply_surrogate<float>(const ApplyArgs<float> &, const float *, int, int, hipStream_t);
template hipError_t launch_apply_surrogate<double>(const ApplyArgs<double> &, const float *, int, int, hipStream_t);
template hipError_t launch_apply_sampled<float>(const ApplyArgs<float> &, const float *, const int *, const int *, int,
                                                hipStream_t);
template hipError_t launch_apply_sampled<double>(const ApplyArgs<double> &, const float *, const int *, const int *,
                                                 int, hipStream_t);

}  // namespace wx
