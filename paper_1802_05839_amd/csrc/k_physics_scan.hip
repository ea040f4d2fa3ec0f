// Column physics with one wavefront per column (lanes = levels, nz <= 64):
// every k-recurrence of the column becomes a wave-wide scan over the lanes
// (shuffles between lanes, log2(64) = 6 combining steps each):
//   * the Thomas forward elimination c'_k = -a_hi / (b_k + a_lo c'_{k-1}) is
//     a chain of Moebius maps, i.e. a prefix product of the 2 x 2 matrices
//     [[0, -a_hi], [a_lo, b_k]] (each partial product rescaled by its largest
//     entry, since only the ratio c' = P01 / P11 matters);
//   * d'_k = (r_k + a_lo d'_{k-1}) / (b_k + a_lo c'_{k-1}) is an affine prefix
//     scan, shared by theta and q (same coefficient, two offsets);
//   * the back substitution delta_k = d'_k - c'_k delta_{k+1} is an affine
//     suffix scan from the lid;
//   * the optical depth tau_{k+1/2} = sum over the levels above k is an
//     exclusive suffix sum.
// The same operations as the thread-per-column kernel in another order, so
// the results agree within rounding, not bit for bit.  Columns whose
// dominance ratio exceeds T_dd run the three scans in FP64 (a wave-uniform
// branch: the whole wave is one column).
//
// Data movement: a block of 256 threads stages 32 neighbouring columns
// (coalesced rows of 32 values per level) of rho, theta, q and the
// cell-centred winds in LDS, each wave then takes 8 of them one after the
// other, and the updated theta and q (or the tendencies) leave through LDS
// again with coalesced stores.
#include "wx_internal.h"

namespace wx {
namespace {

constexpr int SC_COLS = PHYS_SCAN_COLS;   // columns per block
constexpr int SC_LD = 65;                 // LDS row stride (levels), odd: no bank conflicts

template <typename E>
__device__ __forceinline__ E shfl_up_or(E x, int o, E fill) {
  const E y = __shfl_up(x, o, 64);
  return (int(threadIdx.x) & 63) >= o ? y : fill;
}
template <typename E>
__device__ __forceinline__ E shfl_down_or(E x, int o, E fill) {
  const E y = __shfl_down(x, o, 64);
  return (int(threadIdx.x) & 63) + o < 64 ? y : fill;
}
// Lane k - o's value (the identity where there is none) for the six steps
// of a wave-wide inclusive prefix scan built from DPP moves: steps 0-3 shift
// by 1, 2, 4, 8 lanes inside each row of 16, step 4 broadcasts lane 15 of
// rows 0 and 2 to rows 1 and 3, step 5 broadcasts lane 31 to rows 2 and 3.
// After the six steps every lane has combined all lanes below it.
template <int STEP>
__device__ __forceinline__ float dpp_low(float x, float ident) {
  constexpr int ctrl = STEP == 0 ? 0x111 : STEP == 1 ? 0x112 : STEP == 2 ? 0x114 : STEP == 3 ? 0x118
                     : STEP == 4 ? 0x142 : 0x143;
  constexpr int rows = STEP < 4 ? 0xf : STEP == 4 ? 0xa : 0xc;
  return __builtin_amdgcn_update_dpp(ident, x, ctrl, rows, 0xf, false);
}
template <int STEP>
__device__ __forceinline__ double dpp_low(double x, double ident) {
  const long long xv = __double_as_longlong(x), iv = __double_as_longlong(ident);
  constexpr int ctrl = STEP == 0 ? 0x111 : STEP == 1 ? 0x112 : STEP == 2 ? 0x114 : STEP == 3 ? 0x118
                     : STEP == 4 ? 0x142 : 0x143;
  constexpr int rows = STEP < 4 ? 0xf : STEP == 4 ? 0xa : 0xc;
  const int lo = __builtin_amdgcn_update_dpp(int(iv), int(xv), ctrl, rows, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(int(iv >> 32), int(xv >> 32), ctrl, rows, 0xf, false);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

__device__ __forceinline__ float rcp_e(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_e(double x) { return 1.0 / x; }

// Thomas solve of one column for theta and q by scans, lane = level k.
// Inputs per lane: a_lo, a_hi, diag (b_k), right-hand sides rt, rq; lanes at
// or above nz carry the identity.  Returns delta_theta, delta_q.
template <typename E>
__device__ __forceinline__ void scan_solve(bool act, E alo, E ahi, E diag, E rt, E rq, E &dth, E &dqq) {
  // prefix product of the Moebius matrices (high level on the left), six
  // DPP steps
  E p00 = act ? E(0) : E(1), p01 = act ? -ahi : E(0), p10 = act ? alo : E(0), p11 = act ? diag : E(1);
  auto mstep = [&](E q00, E q01, E q10, E q11) {
    const E n00 = p00 * q00 + p01 * q10, n01 = p00 * q01 + p01 * q11;
    const E n10 = p10 * q00 + p11 * q10, n11 = p10 * q01 + p11 * q11;
    const E big = fmax(fmax(fabs(n00), fabs(n01)), fmax(fabs(n10), fabs(n11)));
    const E s = rcp_e(big);
    p00 = n00 * s;
    p01 = n01 * s;
    p10 = n10 * s;
    p11 = n11 * s;
  };
#define WX_MSTEP(S) mstep(dpp_low<S>(p00, E(1)), dpp_low<S>(p01, E(0)), dpp_low<S>(p10, E(0)), dpp_low<S>(p11, E(1)))
  WX_MSTEP(0); WX_MSTEP(1); WX_MSTEP(2); WX_MSTEP(3); WX_MSTEP(4); WX_MSTEP(5);
#undef WX_MSTEP
  const E cp = act ? p01 / p11 : E(0);
  const E cpm = shfl_up_or(cp, 1, E(0));
  const E inv = act ? rcp_e(diag + alo * cpm) : E(0);
  // d'_k = A_k d'_{k-1} + B_k: affine prefix scan (A shared by theta and q)
  E A = act ? alo * inv : E(1), Bt = act ? rt * inv : E(0), Bq = act ? rq * inv : E(0);
  auto astep = [&](E la, E lt, E lq) {
    Bt = A * lt + Bt;
    Bq = A * lq + Bq;
    A = A * la;
  };
#define WX_ASTEP(S) astep(dpp_low<S>(A, E(1)), dpp_low<S>(Bt, E(0)), dpp_low<S>(Bq, E(0)))
  WX_ASTEP(0); WX_ASTEP(1); WX_ASTEP(2); WX_ASTEP(3); WX_ASTEP(4); WX_ASTEP(5);
#undef WX_ASTEP
  // delta_k = -c'_k delta_{k+1} + d'_k: affine suffix scan from the lid
  E C = act ? -cp : E(1), Dt = act ? Bt : E(0), Dq = act ? Bq : E(0);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const E hc = shfl_down_or(C, o, E(1)), ht = shfl_down_or(Dt, o, E(0)), hq = shfl_down_or(Dq, o, E(0));
    Dt = C * ht + Dt;
    Dq = C * hq + Dq;
    C = C * hc;
  }
  dth = Dt;
  dqq = Dq;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_physics_scan(PhysArgs<float> a) {
  __shared__ float sr[SC_COLS * SC_LD], st[SC_COLS * SC_LD], sq[SC_COLS * SC_LD];
  __shared__ float su[SC_COLS * SC_LD], sv[SC_COLS * SC_LD];
  __shared__ double sm[4][6];
  __shared__ int sc[4][3];
  if (a.run_if && *a.run_if == 0) return;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const unsigned sj = a.g.sj, sk = a.g.sk;
  const int nbx = (nx + SC_COLS - 1) / SC_COLS;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int i0 = (L % nbx) * SC_COLS, j = L / nbx;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const unsigned row0 = a.g.origin + unsigned(i0) + unsigned(j) * sj;

  // ---- stage the 32 columns (coalesced rows of 32 values per level)
  for (int e = tid; e < SC_COLS * nz; e += 256) {
    const int c = e % SC_COLS, k = e / SC_COLS;
    if (i0 + c < nx) {
      const unsigned g = row0 + unsigned(c) + unsigned(k) * sk;
      const int o = c * SC_LD + k;
      sr[o] = ldg(a.rho, g);
      st[o] = ldg(a.th, g);
      sq[o] = ldg(a.q, g);
      su[o] = (ldg(a.u, g - 1) + ldg(a.u, g)) * 0.5f;
      sv[o] = (ldg(a.v, g - sj) + ldg(a.v, g)) * 0.5f;
    }
  }
  __syncthreads();

  // per-lane level constants
  const bool act = lane < nz;
  const int k = act ? lane : nz - 1;
  const float dzk = a.dz[k];
  const float rdzi = (lane + 1 < nz) ? a.rdzi[k] : 0.f;
  const double vol = a.vol[k];
  const float dt = a.dt, kmin = a.kmin, l2 = a.l2, kappa = a.kappa, cpa = a.cp;
  Kahan mass[3];
  int nfin = 0, nrho = 0, nfp64 = 0;

  for (int c = wv; c < SC_COLS; c += 4) {
    const int i = i0 + c;
    if (i >= nx) break;                                   // wave-uniform
    const int col = i + nx * j;
    const int o = c * SC_LD + k;
    const float r = sr[o], t = st[o], q = sq[o], ub = su[o], vb = sv[o];
    // level k+1 and k-1 through lane shuffles
    const float r1 = shfl_down_or(r, 1, r), ub1 = shfl_down_or(ub, 1, ub), vb1 = shfl_down_or(vb, 1, vb);
    const float t1 = shfl_down_or(t, 1, t), q1 = shfl_down_or(q, 1, q);
    const float tm = shfl_up_or(t, 1, t), qm = shfl_up_or(q, 1, q);
    float ahi = 0.f;
    if (lane + 1 < nz) {
      const float du = ub1 - ub, dv = vb1 - vb;
      const float kz = kmin + l2 * (__builtin_amdgcn_sqrtf(du * du + dv * dv) * rdzi);
      ahi = dt * ((r + r1) * 0.5f) * kz * rdzi;
    }
    const float alo = shfl_up_or(ahi, 1, 0.f);
    const float m = r * dzk;
    float diag = m + alo + ahi;
    float rt = ahi * (t1 - t) - alo * (t - tm);
    float rq = ahi * (q1 - q) - alo * (q - qm);
    const float beta = dt * __shfl(r, 0, 64) * ldg(a.ch, unsigned(col));
    if (lane == 0) {
      diag += beta;
      rt += beta * (ldg(a.th_s, unsigned(col)) - t);
      rq += beta * (ldg(a.q_s, unsigned(col)) - q);
    }
    // dominance ratio, wave maximum
    float rk = act ? (alo + ahi) * fast_rcp(m) : 0.f;
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) rk = fmaxf(rk, __shfl_xor(rk, s, 64));
    float dth, dqq;
    if (rk > a.tdd) {                                     // wave-uniform
      // FP64 solve from the same FP32 inputs, coefficients rebuilt in FP64
      const double r_ = r, r1_ = r1, ub_ = ub, ub1_ = ub1, vb_ = vb, vb1_ = vb1, t_ = t, q_ = q;
      double ahi_ = 0.0;
      if (lane + 1 < nz) {
        const double du = ub1_ - ub_, dv = vb1_ - vb_;
        const double kz = double(kmin) + double(l2) * (sqrt(du * du + dv * dv) * double(rdzi));
        ahi_ = double(dt) * ((r_ + r1_) * 0.5) * kz * double(rdzi);
      }
      const double alo_ = shfl_up_or(ahi_, 1, 0.0);
      double diag_ = r_ * double(dzk) + alo_ + ahi_;
      double rt_ = ahi_ * (double(t1) - t_) - alo_ * (t_ - double(tm));
      double rq_ = ahi_ * (double(q1) - q_) - alo_ * (q_ - double(qm));
      if (lane == 0) {
        const double beta_ = double(dt) * r_ * double(ldg(a.ch, unsigned(col)));
        diag_ += beta_;
        rt_ += beta_ * (double(ldg(a.th_s, unsigned(col))) - t_);
        rq_ += beta_ * (double(ldg(a.q_s, unsigned(col))) - q_);
      }
      double dt_, dq_;
      scan_solve<double>(act, alo_, ahi_, diag_, rt_, rq_, dt_, dq_);
      dth = float(dt_);
      dqq = float(dq_);
      nfp64 += lane == 0 ? 1 : 0;
    } else {
      scan_solve<float>(act, alo, ahi, diag, rt, rq, dth, dqq);
    }
    // radiation: tau_{k+1/2}, the optical depth of the levels above k, is an
    // exclusive suffix sum from the lid (an inclusive suffix scan of the
    // next level's dtau); the transmissivity below level k is the one above
    // level k-1, taken from that lane, so the fluxes telescope exactly
    const float dtau = act ? kappa * r * (q > 0.f ? q : 0.f) * dzk : 0.f;
    float excl = shfl_down_or(dtau, 1, 0.f);
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) excl += shfl_down_or(excl, s, 0.f);
    const float f0 = ldg(a.f0, unsigned(col));
    const float tr_hi = expf(-excl);
    // (the shuffle runs in every lane: a shuffle inside a lane branch would
    // read the register of a lane that is switched off)
    const float tr_below = shfl_up_or(tr_hi, 1, 1.f);
    const float tr_lo = lane == 0 ? expf(-(excl + dtau)) : tr_below;
    const float heat = f0 * (tr_hi - tr_lo) * fast_rcp(cpa * (r * dzk));
    if (MODE == 1) {
      if (act) {
        st[o] = dth / dt + heat;
        sq[o] = dqq / dt;
      }
    } else {
      const float tn = t + dth + dt * heat;
      const float qn = q + dqq;
      if (act) {
        st[o] = tn;
        sq[o] = qn;
      }
      nfin += (act && !(isfinite(r) && isfinite(tn) && isfinite(qn))) ? 1 : 0;
      nrho += (act && !(r > 0.f)) ? 1 : 0;
      if (a.do_mass) {
        // the column's terms summed over the lanes in a fixed tree, then one
        // compensated add per column
        const double mv = act ? double(r) * vol : 0.0;
        double cm = mv, cmt = mv * (double(tn) + a.theta_off), cmq = mv * double(qn);
        if (!act) cmt = cmq = 0.0;
#pragma unroll
        for (int s = 32; s >= 1; s >>= 1) {
          cm += __shfl_xor(cm, s, 64);
          cmt += __shfl_xor(cmt, s, 64);
          cmq += __shfl_xor(cmq, s, 64);
        }
        if (lane == 0) {
          mass[0].add(cm);
          mass[1].add(cmt);
          mass[2].add(cmq);
        }
      }
    }
  }
  __syncthreads();

  // ---- write back through LDS with coalesced stores (and the periodic
  // images of the state in mode 0)
  for (int e = tid; e < SC_COLS * nz; e += 256) {
    const int c = e % SC_COLS, kk = e / SC_COLS;
    const int i = i0 + c;
    if (i >= nx) continue;
    const int o = c * SC_LD + kk;
    if (MODE == 1) {
      const unsigned fo = unsigned(kk * ny + j) * unsigned(nx) + unsigned(i);
      stg(a.tend_t, fo, st[o]);
      stg(a.tend_q, fo, sq[o]);
    } else {
      const unsigned g = row0 + unsigned(c) + unsigned(kk) * sk;
      const float tn = st[o], qn = sq[o];
      stg(a.th, g, tn);
      stg(a.q, g, qn);
      const int di = i < 2 ? nx : (i >= nx - 2 ? -nx : 0);
      const int dj = j < 2 ? ny * int(sj) : (j >= ny - 2 ? -ny * int(sj) : 0);
      if (di != 0) { stg(a.th, g + di, tn); stg(a.q, g + di, qn); }
      if (dj != 0) {
        stg(a.th, g + dj, tn); stg(a.q, g + dj, qn);
        if (di != 0) { stg(a.th, g + dj + di, tn); stg(a.q, g + dj + di, qn); }
      }
    }
  }

  // ---- block reductions in a fixed order
  if (lane == 0) {
    for (int v = 0; v < 3; ++v) {
      sm[wv][2 * v] = mass[v].s;
      sm[wv][2 * v + 1] = mass[v].c;
    }
  }
  const int nf = wave_sum_int(nfin), nr = wave_sum_int(nrho), nd = wave_sum_int(nfp64);
  if (lane == 0) {
    sc[wv][0] = nf;
    sc[wv][1] = nr;
    sc[wv][2] = nd;
  }
  __syncthreads();
  if (tid == 0) {
    Kahan acc[3];
    int t0 = 0, t1 = 0, t2 = 0;
    for (int w = 0; w < 4; ++w) {
      for (int v = 0; v < 3; ++v) acc[v].merge(sm[w][2 * v], sm[w][2 * v + 1]);
      t0 += sc[w][0];
      t1 += sc[w][1];
      t2 += sc[w][2];
    }
    if (MODE == 0 && a.do_mass) {
      double *p = a.partials + (long long)blockIdx.x * 6;
      for (int v = 0; v < 3; ++v) {
        p[2 * v] = acc[v].s;
        p[2 * v + 1] = acc[v].c;
      }
    }
    if (MODE == 0) {
      if (t0) atomicAdd(&a.flags[0], t0);
      if (t1) atomicAdd(&a.flags[1], t1);
    }
    if (t2) atomicAdd(&a.flags[2], t2);
  }
}

}  // namespace

hipError_t launch_physics_scan(const PhysArgs<float> &a, hipStream_t s) {
  if (a.g.nz > 64 || a.tend_rows || a.col_list) return hipErrorInvalidValue;
  const int nb = phys_scan_blocks(a.g.nx, a.g.ny);
  if (a.mode == 0)
    hipLaunchKernelGGL(k_physics_scan<0>, dim3(nb), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_physics_scan<1>, dim3(nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace wx
