// Surrogate plumbing kernels: per-column feature rows, FP64 normalisation
// statistics, normalisation to the network's input/target form, and batch
// gather.
//
// Feature row of column c = i + nx j (5 nz + 4 values, padded to 320 with
// zeros): five profiles over k = 0..nz-1 built from theta' = theta - 300 K
// (stored value + the state's theta offset - 300, formed in FP64), q and the
// cell-centred winds u = (u_{i-1/2} + u_{i+1/2}) / 2, v likewise: theta'_0 then
// theta' differences; q_0 then q differences; the speed at k = 0 then the
// shear S_k; 0 then S_k times the theta' difference; 0 then S_k times the q
// difference; then theta_s - 300 K, q_s, F0, C_h.  Target row: the 58 theta
// tendencies then the 58 q tendencies, padded to 128.
#include "wx_internal.h"
#include "wx_mlp_internal.h"

namespace wx {
namespace {

constexpr double kThetaRef = 300.0;   // theta features are theta - 300 K

// One thread per column; writes the raw FP32 feature row (mode 0) or the
// normalised BF16 row (mode 1: (x - mean) * inv_std).
template <typename T>
__device__ __forceinline__ LevelVals level_vals(const FeatArgs<T> &a, unsigned g) {
  LevelVals l;
  l.th = float(double(ldg(a.th, g)) + a.theta_off - kThetaRef);
  l.q = float(ldg(a.q, g));
  l.u = float((ldg(a.u, g - 1) + ldg(a.u, g)) * T(0.5));
  l.v = float((ldg(a.v, g - a.g.sj) + ldg(a.v, g)) * T(0.5));
  return l;
}

// One thread per column; writes the raw FP32 feature row (mode 0) or the
// normalised BF16 row (mode 1: (x - mean) * inv_std).
template <typename T>
__global__ void k_features(FeatArgs<T> a) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.nrows) return;
  int c = a.c0 + r;
  if (a.list) c = r < *a.n_list ? a.list[r] : -1;
  if (c < 0) {                                       // unused list slot
    for (int f = 0; f < MLP_KIN; ++f) {
      if (a.mode == 0)
        a.out_f32[(size_t)r * MLP_KIN + f] = 0.f;
      else
        a.out_bf16[(size_t)r * MLP_KIN + f] = 0;
    }
    return;
  }
  const int i = c % a.g.nx, j = c / a.g.nx;
  const unsigned g0 = a.g.origin + unsigned(i) + unsigned(j) * a.g.sj;
  const int nz = a.g.nz;
  auto put = [&](int f, float x) {
    if (a.mode == 0)
      a.out_f32[(size_t)r * MLP_KIN + f] = x;
    else
      a.out_bf16[(size_t)r * MLP_KIN + f] = f2bf((x - a.mean[f]) * a.inv_std[f]);
  };
  LevelVals prev{};
  for (int k = 0; k < nz; ++k) {
    const LevelVals cur = level_vals(a, g0 + unsigned(k) * a.g.sk);
    float fv[5];
    level_features(k, cur, prev, fv);
#pragma unroll
    for (int p = 0; p < 5; ++p) put(p * nz + k, fv[p]);
    prev = cur;
  }
  put(5 * nz, float(double(ldg(a.th_s, unsigned(c))) + a.theta_off - kThetaRef));
  put(5 * nz + 1, float(ldg(a.q_s, unsigned(c))));
  put(5 * nz + 2, float(ldg(a.f0, unsigned(c))));
  put(5 * nz + 3, float(ldg(a.ch, unsigned(c))));
  for (int f = 5 * nz + 4; f < MLP_KIN; ++f) {
    if (a.mode == 0)
      a.out_f32[(size_t)r * MLP_KIN + f] = 0.f;
    else
      a.out_bf16[(size_t)r * MLP_KIN + f] = 0;
  }
}

// FP64 column statistics of an [n][ld] FP32 matrix, two levels in a fixed
// order: chunk partial sums (of x, or of (x - mean)^2 when mean != null).
__global__ void k_stat_part(const float *x, size_t n, int ld, int cols, size_t chunk, const double *mean,
                            double *part) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= cols) return;
  const size_t r0 = size_t(blockIdx.y) * chunk, r1 = min(n, r0 + chunk);
  double s = 0.0;
  const double mu = mean ? mean[col] : 0.0;
  for (size_t r = r0; r < r1; ++r) {
    const double v = double(x[r * ld + col]);
    s += mean ? (v - mu) * (v - mu) : v;
  }
  part[size_t(blockIdx.y) * cols + col] = s;
}

__global__ void k_stat_fold(const double *part, int nchunk, int cols, double scale, double *out) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= cols) return;
  double s = 0.0;
  for (int p = 0; p < nchunk; ++p) s += part[size_t(p) * cols + col];
  out[col] = s * scale;
}

// Statistics to the blob: feature mean and 1 / std, target mean per output,
// and the pooled std of the theta and q tendencies from the per-output
// statistics, sigma_v^2 = mean over the 58 outputs of (var_o + (mean_o -
// pooled_mean)^2), which also scales every target of that variable.
__global__ void k_norm_finish(const double *xmean, const double *xvar, const double *ymean, const double *yvar,
                              int nin, int nout, float *xm, float *xis, float *ym, float *ys, float *sig,
                              double *sig64) {
  const int t = threadIdx.x;
  for (int f = t; f < MLP_KIN; f += blockDim.x) {
    if (f < nin) {
      const double sd = sqrt(xvar[f]);
      xm[f] = float(xmean[f]);
      xis[f] = float(1.0 / (sd < 1e-12 ? 1.0 : sd));
    } else {
      xm[f] = 0.f;
      xis[f] = 0.f;
    }
  }
  // pooled std of each variable (every thread computes both, same order)
  const int h = nout / 2;
  double pooled[2];
  for (int var = 0; var < 2; ++var) {
    const int o0 = var * h;
    double mu = 0.0;
    for (int o = 0; o < h; ++o) mu += ymean[o0 + o];
    mu /= h;
    double v = 0.0;
    for (int o = 0; o < h; ++o) v += yvar[o0 + o] + (ymean[o0 + o] - mu) * (ymean[o0 + o] - mu);
    pooled[var] = sqrt(v / h);
  }
  for (int o = t; o < MLP_NOUTP; o += blockDim.x) {
    if (o < nout) {
      const double sd = pooled[o < h ? 0 : 1];
      ym[o] = float(ymean[o]);
      ys[o] = float(sd < 1e-12 ? 1.0 : sd);
    } else {
      ym[o] = 0.f;
      ys[o] = 1.f;
    }
  }
  if (t < 2) {
    sig64[t] = pooled[t];
    sig[t] = float(pooled[t]);
  }
}

__global__ void k_normalize(const float *xr, const float *yr, size_t n, const float *xm, const float *xis,
                            const float *ym, const float *ys, uint16_t *xo, float *yo) {
  const size_t r = blockIdx.x;
  for (int f = threadIdx.x; f < MLP_KIN; f += blockDim.x)
    xo[r * MLP_KIN + f] = f2bf((xr[r * MLP_KIN + f] - xm[f]) * xis[f]);
  if (yr)
    for (int o = threadIdx.x; o < MLP_NOUTP; o += blockDim.x)
      yo[r * MLP_NOUTP + o] = o < MLP_NOUT ? (yr[r * MLP_NOUTP + o] - ym[o]) / ys[o] : 0.f;
}

}  // namespace

template <typename T>
hipError_t launch_features(const FeatArgs<T> &a, hipStream_t s) {
  if (a.nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_features<T>, dim3((a.nrows + 127) / 128), dim3(128), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fit_norm(const float *xr, const float *yr, size_t n, double *scratch, float *xm, float *xis,
                           float *ym, float *ys, float *sig, double *sig64, hipStream_t s) {
  const size_t chunk = 4096;
  const int nchunk = int((n + chunk - 1) / chunk);
  double *part = scratch;                                   // nchunk * 320
  double *xmean = part + size_t(nchunk) * MLP_KIN, *xvar = xmean + MLP_KIN;
  double *ymean = xvar + MLP_KIN, *yvar = ymean + MLP_NOUTP;
  const double inv = 1.0 / double(n);
  hipLaunchKernelGGL(k_stat_part, dim3((MLP_KIN + 63) / 64, nchunk), dim3(64), 0, s, xr, n, MLP_KIN, MLP_KIN, chunk,
                     (const double *)nullptr, part);
  hipLaunchKernelGGL(k_stat_fold, dim3((MLP_KIN + 63) / 64), dim3(64), 0, s, part, nchunk, MLP_KIN, inv, xmean);
  hipLaunchKernelGGL(k_stat_part, dim3((MLP_KIN + 63) / 64, nchunk), dim3(64), 0, s, xr, n, MLP_KIN, MLP_KIN, chunk,
                     (const double *)xmean, part);
  hipLaunchKernelGGL(k_stat_fold, dim3((MLP_KIN + 63) / 64), dim3(64), 0, s, part, nchunk, MLP_KIN, inv, xvar);
  hipLaunchKernelGGL(k_stat_part, dim3((MLP_NOUTP + 63) / 64, nchunk), dim3(64), 0, s, yr, n, MLP_NOUTP, MLP_NOUTP,
                     chunk, (const double *)nullptr, part);
  hipLaunchKernelGGL(k_stat_fold, dim3((MLP_NOUTP + 63) / 64), dim3(64), 0, s, part, nchunk, MLP_NOUTP, inv, ymean);
  hipLaunchKernelGGL(k_stat_part, dim3((MLP_NOUTP + 63) / 64, nchunk), dim3(64), 0, s, yr, n, MLP_NOUTP, MLP_NOUTP,
                     chunk, (const double *)ymean, part);
  hipLaunchKernelGGL(k_stat_fold, dim3((MLP_NOUTP + 63) / 64), dim3(64), 0, s, part, nchunk, MLP_NOUTP, inv, yvar);
  hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(128), 0, s, xmean, xvar, ymean, yvar, MLP_NIN, MLP_NOUT, xm, xis, ym,
                     ys, sig, sig64);
  return hipGetLastError();
}

size_t fit_norm_scratch_bytes(size_t n) {
  const size_t nchunk = (n + 4095) / 4096;
  return (nchunk * MLP_KIN + 2 * MLP_KIN + 2 * MLP_NOUTP) * sizeof(double);
}

hipError_t launch_normalize(const float *xr, const float *yr, size_t n, const float *xm, const float *xis,
                            const float *ym, const float *ys, uint16_t *xo, float *yo, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_normalize, dim3(unsigned(n)), dim3(128), 0, s, xr, yr, n, xm, xis, ym, ys, xo, yo);
  return hipGetLastError();
}

template hipError_t launch_features<float>(const FeatArgs<float> &, hipStream_t);
template hipError_t launch_features<double>(const FeatArgs<double> &, hipStream_t);

}  // namespace wx
