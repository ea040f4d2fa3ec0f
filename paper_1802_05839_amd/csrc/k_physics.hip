// Column physics and global mass sums.
//
// Method (readings; the paper fixes only that physics runs column by column
// after the dycore, sequential in K, without horizontal communication --
// sections "Architecture-Dependant Parallelization Granularity" and "The
// ASUCA Weather Prediction Model" -- and that radiation and boundary-layer
// physics are the processes that matter, section "Hybrid ASUCA Strong Scaling
// GPU Results"):
//   K_{k+1/2}   = K_min + l^2 |U_{k+1} - U_k| / dz_{k+1/2}   (cell-centred winds)
//   alpha_{k+1/2} = dt rho_{k+1/2} K / dz_{k+1/2};  m_k = rho_k dz_k;  beta = dt rho_0 C_h
//   delta form:  -alpha_lo d_{k-1} + (m_k + alpha_lo + alpha_hi [+ beta]) d_k - alpha_hi d_{k+1}
//                = alpha_hi (phi_{k+1} - phi_k) - alpha_lo (phi_k - phi_{k-1}) [+ beta (phi_s - phi_0)]
//   radiation:   dtau_k = kappa rho_k max(q_k, 0) dz_k, tau summed from the lid down,
//                H_k = F0 (exp(-tau_{k+1/2}) - exp(-tau_{k-1/2})) / (c_p m_k)
//   update:      theta += d_theta + dt H,  q += d_q.
//
// GPU design: one thread per column, 64 columns (one wave) per block, i
// coalesced.  The upward pass reads each level once, builds the matrix row
// from a one-level look-ahead and does the Thomas forward elimination for
// theta and q together (shared matrix), keeping c', d'_theta, d'_q in LDS.
// The downward pass back-substitutes, accumulates the optical depth from the
// lid (the suffix sum) and writes the new state.  A column whose dominance
// ratio max_k (alpha_lo + alpha_hi) / m_k exceeds T_dd repeats the forward
// elimination in FP64 (coefficients rebuilt in FP64 from the same inputs) with
// its c'/d' in a global scratch; such columns are counted.  The epilogue
// accumulates the compensated FP64 mass sums (Neumaier) and the fault
// counters; blocks reduce them in a fixed order.
#include "wx_internal.h"

namespace wx {
namespace {

struct Kahan {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
    s = t;
  }
  __device__ __forceinline__ void merge(double s2, double c2) {
    const double t = s + s2;
    c += c2 + ((fabs(s) >= fabs(s2)) ? ((s - t) + s2) : ((s2 - t) + s));
    s = t;
  }
};

// Fixed-order reduction over the 64 lanes of a wave; lane 0 holds the result.
__device__ __forceinline__ void wave_merge(Kahan &k) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double s2 = __shfl_down(k.s, off, 64);
    const double c2 = __shfl_down(k.c, off, 64);
    k.merge(s2, c2);
  }
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// c', d'_theta, d'_q storage: LDS [3][nz][64] or global [3][nz][ncol].
template <typename E>
struct LdsStore {
  E *p;
  int nz, lane;
  __device__ __forceinline__ E &at(int v, int k) const { return p[(v * nz + k) * PHYS_BX + lane]; }
};
template <typename E>
struct GlobalStore {
  E *p;
  int nz;
  long long ncol, col;
  __device__ __forceinline__ E &at(int v, int k) const { return p[((long long)v * nz + k) * ncol + col]; }
};

template <typename T>
struct Column {
  const PhysArgs<T> &a;
  long long g0;     // element offset of level 0 of this column
  int col;          // i + nx j
  __device__ __forceinline__ long long at(int k) const { return g0 + (long long)k * a.g.sk; }
};

// Forward elimination (bottom to top) in precision E.  Returns max_k r_k.
template <typename T, typename E, typename S>
__device__ T upward(const Column<T> &c, const S &st) {
  const PhysArgs<T> &a = c.a;
  const int nz = a.g.nz;
  const long long sj = a.g.sj;
  const E dt = E(a.dt), kmin = E(a.kmin), l2 = E(a.l2);
  long long g = c.at(0);
  E r0 = E(a.rho[g]), t0 = E(a.th[g]), q0 = E(a.q[g]);
  E ub0 = (E(a.u[g - 1]) + E(a.u[g])) * E(0.5);
  E vb0 = (E(a.v[g - sj]) + E(a.v[g])) * E(0.5);
  const E beta = dt * r0 * E(a.ch[c.col]);
  const E ths = E(a.th_s[c.col]), qs = E(a.q_s[c.col]);
  E alo = 0, tm1 = t0, qm1 = q0;
  E cp = 0, dtp = 0, dqp = 0;
  T rmax = T(0);
  for (int k = 0; k < nz; ++k) {
    E ahi = 0, r1 = 0, t1 = t0, q1 = q0, ub1 = 0, vb1 = 0;
    if (k + 1 < nz) {
      g = c.at(k + 1);
      r1 = E(a.rho[g]);
      t1 = E(a.th[g]);
      q1 = E(a.q[g]);
      ub1 = (E(a.u[g - 1]) + E(a.u[g])) * E(0.5);
      vb1 = (E(a.v[g - sj]) + E(a.v[g])) * E(0.5);
      const E rdzi = E(a.rdzi[k]);
      const E du = ub1 - ub0, dv = vb1 - vb0;
      const E kz = kmin + l2 * (sqrt(du * du + dv * dv) * rdzi);
      ahi = dt * ((r0 + r1) * E(0.5)) * kz * rdzi;
    }
    const E m = r0 * E(a.dz[k]);
    E diag = m + alo + ahi;
    E rt = ahi * (t1 - t0) - alo * (t0 - tm1);
    E rq = ahi * (q1 - q0) - alo * (q0 - qm1);
    if (k == 0) {
      diag += beta;
      rt += beta * (ths - t0);
      rq += beta * (qs - q0);
    }
    const T rk = T((alo + ahi) / m);
    rmax = rk > rmax ? rk : rmax;
    const E inv = E(1) / (diag + alo * cp);
    cp = -ahi * inv;
    dtp = (rt + alo * dtp) * inv;
    dqp = (rq + alo * dqp) * inv;
    st.at(0, k) = cp;
    st.at(1, k) = dtp;
    st.at(2, k) = dqp;
    alo = ahi;
    tm1 = t0; t0 = t1;
    qm1 = q0; q0 = q1;
    r0 = r1; ub0 = ub1; vb0 = vb1;
  }
  return rmax;
}

struct Counters {
  int nonfinite = 0, rho_le0 = 0;
};

// Back substitution (top to bottom), radiation suffix scan and the update.
template <typename T, typename E, typename S>
__device__ void downward(const Column<T> &c, const S &st, Kahan *mass, Counters &cnt) {
  const PhysArgs<T> &a = c.a;
  const int nz = a.g.nz;
  const T f0 = a.f0[c.col];
  const T kappa = a.kappa, cpa = a.cp, dt = a.dt;
  const int i = c.col % a.g.nx, j = c.col / a.g.nx;
  const int nx = a.g.nx, ny = a.g.ny;
  const long long di = i < 2 ? nx : (i >= nx - 2 ? -nx : 0);
  const long long dj = j < 2 ? (long long)ny * a.g.sj : (j >= ny - 2 ? -(long long)ny * a.g.sj : 0);
  E dtn = 0, dqn = 0;
  T tau = T(0), tr_hi = T(1);
  for (int k = nz - 1; k >= 0; --k) {
    const E dth = st.at(1, k) - st.at(0, k) * dtn;
    const E dqq = st.at(2, k) - st.at(0, k) * dqn;
    dtn = dth;
    dqn = dqq;
    const long long g = c.at(k);
    const T r = a.rho[g], t = a.th[g], q = a.q[g];
    const T dzk = a.dz[k];
    tau += kappa * r * (q > T(0) ? q : T(0)) * dzk;
    const T tr_lo = exp(-tau);
    const T heat = f0 * (tr_hi - tr_lo) / (cpa * (r * dzk));
    tr_hi = tr_lo;
    if (a.mode == 1) {
      const long long o = ((long long)k * ny + j) * nx + i;
      a.tend_t[o] = T(dth) / dt + heat;
      a.tend_q[o] = T(dqq) / dt;
      continue;
    }
    const T tn = t + T(dth) + dt * heat;
    const T qn = q + T(dqq);
    a.th[g] = tn;
    a.q[g] = qn;
    if (di != 0) { a.th[g + di] = tn; a.q[g + di] = qn; }
    if (dj != 0) {
      a.th[g + dj] = tn; a.q[g + dj] = qn;
      if (di != 0) { a.th[g + dj + di] = tn; a.q[g + dj + di] = qn; }
    }
    if (!(isfinite(r) && isfinite(tn) && isfinite(qn))) cnt.nonfinite++;
    if (!(r > T(0))) cnt.rho_le0++;
    if (a.do_mass) {
      const double mv = double(r) * a.vol[k];
      mass[0].add(mv);
      mass[1].add(mv * (double(tn) + a.theta_off));
      mass[2].add(mv * double(qn));
    }
  }
}

template <typename T>
__global__ __launch_bounds__(PHYS_BX) void k_physics(PhysArgs<T> a) {
  extern __shared__ unsigned char s_raw[];
  const int nbx = (a.g.nx + PHYS_BX - 1) / PHYS_BX;
  const int bi = blockIdx.x % nbx, j = blockIdx.x / nbx;
  const int lane = threadIdx.x;
  const int i = bi * PHYS_BX + lane;
  const bool active = i < a.g.nx;
  Kahan mass[3];
  Counters cnt;
  int fp64 = 0;
  if (active) {
    const Column<T> c{a, a.g.origin + i + (long long)j * a.g.sj, i + a.g.nx * j};
    const long long ncol = (long long)a.g.nx * a.g.ny;
    bool wide;
    if (sizeof(T) == 4) {
      if (a.use_lds) {
        const LdsStore<float> st{reinterpret_cast<float *>(s_raw), a.g.nz, lane};
        wide = upward<T, float>(c, st) > a.tdd;
        if (!wide) downward<T, float>(c, st, mass, cnt);
      } else {
        const GlobalStore<float> st{reinterpret_cast<float *>(a.scratch), a.g.nz, ncol, c.col};
        wide = upward<T, float>(c, st) > a.tdd;
        if (!wide) downward<T, float>(c, st, mass, cnt);
      }
    } else {
      const GlobalStore<double> st{a.scratch, a.g.nz, ncol, c.col};
      wide = upward<T, double>(c, st) > a.tdd;
      downward<T, double>(c, st, mass, cnt);
      fp64 = wide ? 1 : 0;
      wide = false;
    }
    if (wide) {
      const GlobalStore<double> st{a.scratch, a.g.nz, ncol, c.col};
      upward<T, double>(c, st);
      downward<T, double>(c, st, mass, cnt);
      fp64 = 1;
    }
  }
  // block (= one wave) reductions in a fixed order
  const int nf = wave_sum_i(cnt.nonfinite), nr = wave_sum_i(cnt.rho_le0), nd = wave_sum_i(fp64);
  if (a.mode == 0 && a.do_mass) {
    for (int v = 0; v < 3; ++v) wave_merge(mass[v]);
    if (lane == 0) {
      double *p = a.partials + (long long)blockIdx.x * 6;
      for (int v = 0; v < 3; ++v) {
        p[2 * v] = mass[v].s;
        p[2 * v + 1] = mass[v].c;
      }
    }
  }
  if (lane == 0 && a.mode == 0) {
    if (nf) atomicAdd(&a.flags[0], nf);
    if (nr) atomicAdd(&a.flags[1], nr);
  }
  if (lane == 0 && nd) atomicAdd(&a.flags[2], nd);
}

template <typename T>
__global__ __launch_bounds__(PHYS_BX) void k_mass(MassArgs<T> a) {
  const int nbx = (a.g.nx + PHYS_BX - 1) / PHYS_BX;
  const int bi = blockIdx.x % nbx, j = blockIdx.x / nbx;
  const int lane = threadIdx.x;
  const int i = bi * PHYS_BX + lane;
  Kahan mass[3];
  Counters cnt;
  if (i < a.g.nx) {
    const long long g0 = a.g.origin + i + (long long)j * a.g.sj;
    for (int k = 0; k < a.g.nz; ++k) {
      const long long g = g0 + (long long)k * a.g.sk;
      const T r = a.rho[g], t = a.th[g], q = a.q[g];
      if (!(isfinite(r) && isfinite(t) && isfinite(q))) cnt.nonfinite++;
      if (!(r > T(0))) cnt.rho_le0++;
      const double mv = double(r) * a.vol[k];
      mass[0].add(mv);
      mass[1].add(mv * (double(t) + a.theta_off));
      mass[2].add(mv * double(q));
    }
  }
  for (int v = 0; v < 3; ++v) wave_merge(mass[v]);
  const int nf = wave_sum_i(cnt.nonfinite), nr = wave_sum_i(cnt.rho_le0);
  if (lane == 0) {
    double *p = a.partials + (long long)blockIdx.x * 6;
    for (int v = 0; v < 3; ++v) {
      p[2 * v] = mass[v].s;
      p[2 * v + 1] = mass[v].c;
    }
    if (nf) atomicAdd(&a.flags[0], nf);
    if (nr) atomicAdd(&a.flags[1], nr);
  }
}

// One block: thread t folds partials t, t+256, ... in order, then a fixed tree.
__global__ __launch_bounds__(256) void k_mass_final(const double *parts, int n, double *out) {
  __shared__ double sh[6][256];
  const int t = threadIdx.x;
  Kahan acc[3];
  for (int b = t; b < n; b += 256)
    for (int v = 0; v < 3; ++v) acc[v].merge(parts[(long long)b * 6 + 2 * v], parts[(long long)b * 6 + 2 * v + 1]);
  for (int v = 0; v < 3; ++v) {
    sh[2 * v][t] = acc[v].s;
    sh[2 * v + 1][t] = acc[v].c;
  }
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (t < w) {
      for (int v = 0; v < 3; ++v) {
        Kahan k;
        k.s = sh[2 * v][t];
        k.c = sh[2 * v + 1][t];
        k.merge(sh[2 * v][t + w], sh[2 * v + 1][t + w]);
        sh[2 * v][t] = k.s;
        sh[2 * v + 1][t] = k.c;
      }
    }
    __syncthreads();
  }
  if (t < 6) out[t] = sh[t][0];
}

__global__ void k_fill_i32(int *p, int n, int value) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = value;
}

__global__ void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) dst[t] = src[t];
}

}  // namespace

template <typename T>
hipError_t launch_physics(const PhysArgs<T> &a, hipStream_t s) {
  const int nb = phys_blocks(a.g.nx, a.g.ny);
  const size_t lds = (sizeof(T) == 4 && a.use_lds) ? size_t(3) * a.g.nz * PHYS_BX * sizeof(float) : 0;
  hipLaunchKernelGGL(k_physics<T>, dim3(nb), dim3(PHYS_BX), lds, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mass(const MassArgs<T> &a, hipStream_t s) {
  hipLaunchKernelGGL(k_mass<T>, dim3(phys_blocks(a.g.nx, a.g.ny)), dim3(PHYS_BX), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mass_final(const double *partials, int nparts, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(256), 0, s, partials, nparts, out);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int *p, int n, int value, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, value);
  return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s) {
  const long long n = (long long)(bytes / 16);
  long long blocks = (n + 255) / 256;
  if (blocks > 1 << 20) blocks = 1 << 20;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s,
                     reinterpret_cast<const uint4 *>(src), reinterpret_cast<uint4 *>(dst), n);
  return hipGetLastError();
}

template hipError_t launch_physics<float>(const PhysArgs<float> &, hipStream_t);
template hipError_t launch_physics<double>(const PhysArgs<double> &, hipStream_t);
template hipError_t launch_mass<float>(const MassArgs<float> &, hipStream_t);
template hipError_t launch_mass<double>(const MassArgs<double> &, hipStream_t);

}  // namespace wx
