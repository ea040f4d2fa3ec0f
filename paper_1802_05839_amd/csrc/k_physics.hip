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


// Fixed-order reduction over the 64 lanes of a wave; lane 0 holds the result.
__device__ __forceinline__ void wave_merge(Kahan &k) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double s2 = __shfl_down(k.s, off, 64);
    const double c2 = __shfl_down(k.c, off, 64);
    k.merge(s2, c2);
  }
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
  unsigned ncol, col;
  __device__ __forceinline__ E &at(int v, int k) const { return ref(p, unsigned(v * nz + k) * ncol + col); }
};

template <typename T>
struct Column {
  const PhysArgs<T> &a;
  unsigned g0;      // element offset of level 0 of this column
  int col;          // i + nx j
  int row;          // output row of the row-major tendency layout
  __device__ __forceinline__ unsigned at(int k) const { return g0 + unsigned(k) * a.g.sk; }
};

// Forward elimination (bottom to top) in precision E.  Returns max_k r_k.
template <typename T, typename E, int NZC, typename S>
__device__ __forceinline__ T upward(const Column<T> &c, const S &st) {
  const PhysArgs<T> &a = c.a;
  const int nz = NZC > 0 ? NZC : a.g.nz;
  const unsigned sj = a.g.sj;
  const E dt = E(a.dt), kmin = E(a.kmin), l2 = E(a.l2);
  unsigned g = c.at(0);
  E r0 = E(ldg(a.rho, g)), t0 = E(ldg(a.th, g)), q0 = E(ldg(a.q, g));
  E ub0 = (E(ldg(a.u, g - 1)) + E(ldg(a.u, g))) * E(0.5);
  E vb0 = (E(ldg(a.v, g - sj)) + E(ldg(a.v, g))) * E(0.5);
  const E beta = dt * r0 * E(a.ch[c.col]);
  const E ths = E(a.th_s[c.col]), qs = E(a.q_s[c.col]);
  E alo = 0, tm1 = t0, qm1 = q0;
  E cp = 0, dtp = 0, dqp = 0;
  T rmax = T(0);
#pragma unroll
  for (int k = 0; k < nz; ++k) {
    E ahi = 0, r1 = 0, t1 = t0, q1 = q0, ub1 = 0, vb1 = 0;
    if (k + 1 < nz) {
      g = c.at(k + 1);
      r1 = E(ldg(a.rho, g));
      t1 = E(ldg(a.th, g));
      q1 = E(ldg(a.q, g));
      ub1 = (E(ldg(a.u, g - 1)) + E(ldg(a.u, g))) * E(0.5);
      vb1 = (E(ldg(a.v, g - sj)) + E(ldg(a.v, g))) * E(0.5);
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
    const T rk = T((alo + ahi) * fast_rcp(m));
    rmax = rk > rmax ? rk : rmax;
    const E inv = fast_rcp(diag + alo * cp);
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
    // keep each level's loads next to their use when the loop is unrolled
    // (otherwise all levels' loads are hoisted and the registers spill)
    if (NZC > 0) __builtin_amdgcn_sched_barrier(0);
  }
  return rmax;
}

struct Counters {
  int nonfinite = 0, rho_le0 = 0;
};

// Back substitution (top to bottom), radiation suffix scan and the update.
template <typename T, typename E, int NZC, int MODE, typename S>
__device__ __forceinline__ void downward(const Column<T> &c, const S &st, Kahan *mass, Counters &cnt) {
  const PhysArgs<T> &a = c.a;
  const int nz = NZC > 0 ? NZC : a.g.nz;
  const T f0 = a.f0[c.col];
  const T kappa = a.kappa, cpa = a.cp, dt = a.dt;
  const int i = c.col % a.g.nx, j = c.col / a.g.nx;
  const int nx = a.g.nx, ny = a.g.ny;
  const int di = i < 2 ? nx : (i >= nx - 2 ? -nx : 0);
  const int dj = j < 2 ? ny * int(a.g.sj) : (j >= ny - 2 ? -ny * int(a.g.sj) : 0);
  E dtn = 0, dqn = 0;
  T tau = T(0), tr_hi = T(1);
#pragma unroll
  for (int k = nz - 1; k >= 0; --k) {
    const E dth = st.at(1, k) - st.at(0, k) * dtn;
    const E dqq = st.at(2, k) - st.at(0, k) * dqn;
    dtn = dth;
    dqn = dqq;
    const unsigned g = c.at(k);
    const T r = ldg(a.rho, g), t = ldg(a.th, g), q = ldg(a.q, g);
    const T dzk = a.dz[k];
    tau += kappa * r * (q > T(0) ? q : T(0)) * dzk;
    const T tr_lo = exp(-tau);
    const T heat = f0 * (tr_hi - tr_lo) * fast_rcp(cpa * (r * dzk));
    tr_hi = tr_lo;
    if (MODE == 1) {
      if (a.tend_rows) {
        const unsigned o = unsigned(c.row) * TEND_ROW + unsigned(k);
        stg(a.tend_t, o, T(dth) / dt + heat);
        stg(a.tend_t, o + unsigned(nz), T(dqq) / dt);
        if (k == 0)
          for (int p = 2 * nz; p < TEND_ROW; ++p) stg(a.tend_t, unsigned(c.row) * TEND_ROW + unsigned(p), T(0));
      } else {
        const unsigned o = unsigned(k * ny + j) * unsigned(nx) + unsigned(i);
        stg(a.tend_t, o, T(dth) / dt + heat);
        stg(a.tend_q, o, T(dqq) / dt);
      }
      if (NZC > 0) __builtin_amdgcn_sched_barrier(0);
      continue;
    }
    const T tn = t + T(dth) + dt * heat;
    const T qn = q + T(dqq);
    stg(a.th, g, tn);
    stg(a.q, g, qn);
    if (di != 0) { stg(a.th, g + di, tn); stg(a.q, g + di, qn); }
    if (dj != 0) {
      stg(a.th, g + dj, tn); stg(a.q, g + dj, qn);
      if (di != 0) { stg(a.th, g + dj + di, tn); stg(a.q, g + dj + di, qn); }
    }
    if (!(isfinite(r) && isfinite(tn) && isfinite(qn))) cnt.nonfinite++;
    if (!(r > T(0))) cnt.rho_le0++;
    if (a.do_mass) {
      const double mv = double(r) * a.vol[k];
      mass[0].add(mv);
      mass[1].add(mv * (double(tn) + a.theta_off));
      mass[2].add(mv * double(qn));
    }
    if (NZC > 0) __builtin_amdgcn_sched_barrier(0);
  }
}


// Fixed-order block reduction of the per-wave results (waves 0..NW-1).
template <int NW>
__device__ __forceinline__ void block_finish(const PhysArgs<float> *ap, double *partials, int *flags,
                                             bool do_mass, bool count_faults, Kahan *mass,
                                             const Counters &cnt, int fp64) {
  __shared__ double sm[NW][6];
  __shared__ int sc[NW][3];
  const int tid = threadIdx.x + threadIdx.y * blockDim.x;
  const int lane = tid & 63, wv = tid >> 6;
  (void)ap;
  const int nf = wave_sum_int(cnt.nonfinite), nr = wave_sum_int(cnt.rho_le0), nd = wave_sum_int(fp64);
  if (do_mass)
    for (int v = 0; v < 3; ++v) wave_merge(mass[v]);
  if (lane == 0) {
    for (int v = 0; v < 3; ++v) {
      sm[wv][2 * v] = mass[v].s;
      sm[wv][2 * v + 1] = mass[v].c;
    }
    sc[wv][0] = nf;
    sc[wv][1] = nr;
    sc[wv][2] = nd;
  }
  __syncthreads();
  if (tid == 0) {
    Kahan acc[3];
    int t0 = 0, t1 = 0, t2 = 0;
    for (int w = 0; w < NW; ++w) {
      for (int v = 0; v < 3; ++v) acc[v].merge(sm[w][2 * v], sm[w][2 * v + 1]);
      t0 += sc[w][0];
      t1 += sc[w][1];
      t2 += sc[w][2];
    }
    if (do_mass) {
      double *p = partials + (long long)blockIdx.x * 6;
      for (int v = 0; v < 3; ++v) {
        p[2 * v] = acc[v].s;
        p[2 * v + 1] = acc[v].c;
      }
    }
    if (count_faults) {
      if (t0) atomicAdd(&flags[0], t0);
      if (t1) atomicAdd(&flags[1], t1);
    }
    if (t2) atomicAdd(&flags[2], t2);
  }
}

// FP32 state with a compile-time level count NZ, one thread per column (the
// two-lane kernel below is the default; these are its ablation variants).
//
// 64 x 4 columns per block, one thread per column.  The forward elimination
// keeps c' in LDS (one float per level and column) and d'_theta, d'_q and the
// column's rho, theta, q in registers (every loop over k is unrolled, so each
// array element is a fixed register), so the downward pass reads nothing from
// HBM.  The upward pass prefetches the inputs of level k + PF while working on
// level k (a register ring of PF levels), so a wave never waits on the load it
// is about to use; a scheduling barrier per level keeps the compiler from
// hoisting further and running out of registers.  Columns whose dominance
// ratio exceeds T_dd redo the elimination in FP64 (runtime loop, global
// scratch).
//
// KEEP = false is the variant that does not keep the column in registers: the
// downward pass reads rho, theta, q again (the same block read them a moment
// earlier, so they come from the caches, not HBM) through a prefetch ring of
// its own.  That halves the registers, so two waves share each SIMD and one
// wave's loads overlap the other's arithmetic.
//
// WIDE (with KEEP) is the variant whose upward pass fetches a level with two
// 16-byte loads per lane instead of seven 4-byte ones: a wave loads its row's
// columns i0-2 .. i0+65 of rho, theta, q, u, v and of v in row j-1 (17
// aligned 16-byte chunks each), writes them to its own LDS slot and reads its
// column back (LDS runs a wave's accesses in order: no barrier).  At one wave
// per SIMD the number of vector-memory instructions a wave keeps in flight,
// not their size, bounds the bandwidth, so 16-byte loads move about four
// times as much.  Whole waves take part in the loads: a lane past the grid
// edge works on column nx-1 (the same values and the same stores as the lane
// that owns it) and counts nothing.
template <int NZ, int MODE, bool KEEP, bool WIDE = false>
__global__ __launch_bounds__(256, KEEP ? 1 : 2) void k_physics_f32(PhysArgs<float> a) {
  static_assert(!WIDE || KEEP, "the wide upward pass keeps the column in registers");
  constexpr int PF = KEEP ? 8 : 4;     // levels prefetched ahead (two waves per SIMD need half)
  constexpr int WROW = 68, WSLOT = WIDE ? 6 * WROW : 1;   // floats per field row and per wave slot
  __shared__ __attribute__((aligned(16))) float s_w[4][WSLOT];
  extern __shared__ float s_c[];          // [NZ][256]
  // the per-level constants, staged once per block: read through LDS they
  // never wait behind the kernel's own global stores (on this target the
  // vector-memory counter tracks stores too, and vector loads of these
  // read-only arrays would drain it every level)
  __shared__ float s_dz[NZ], s_rdzi[NZ];
  __shared__ double s_vol[NZ];
  if (a.run_if && *a.run_if == 0) return;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 64 + tx;
  for (int k = tid; k < NZ; k += 256) {
    s_dz[k] = a.dz[k];
    s_rdzi[k] = k + 1 < NZ ? a.rdzi[k] : 0.f;
    s_vol[k] = a.vol[k];
  }
  __syncthreads();
  const int nbx = (a.g.nx + 63) / 64;
  const int L = xcd_remap(blockIdx.x, gridDim.x);   // j-neighbours share an XCD's L2 (the v row below)
  const int i0 = (L % nbx) * 64, i = i0 + tx, j = (L / nbx) * 4 + ty;
  const bool active = (i < a.g.nx) && (j < a.g.ny);
  // WIDE: the whole wave of a row inside the grid runs, on column min(i, nx-1)
  const bool run = WIDE ? (j < a.g.ny) : active;
  const int ic = WIDE ? min(i, a.g.nx - 1) : i;
  Kahan mass[3];
  Counters cnt;
  int fp64 = 0;
  if (run) {
    const unsigned sj = a.g.sj, sk = a.g.sk;
    const unsigned g0 = a.g.origin + unsigned(ic) + unsigned(j) * sj;
    const int col = ic + a.g.nx * j;
    const float dt = a.dt, kmin = a.kmin, l2 = a.l2;

    // ---- upward pass: build row k from a one-level look-ahead, eliminate
    float pr[PF], pt[PF], pq[PF], pu[PF], pe[PF], pv[PF], pn[PF];  // prefetch ring, levels k+1 .. k+PF
    // west and south face winds through shifted (uniform) base pointers, so
    // that all seven loads of a level share one vector offset
    const float *uw = plane(a.u, -1), *vs = plane(a.v, -(long long)sj);
    // per-level offsets are made opaque (asm) so that the compiler forms each
    // where it is used instead of all NZ of them up front in registers
    auto fetch_up = [&](int lev, int slot) {
      unsigned g = g0 + unsigned(lev) * sk;
      asm volatile("" : "+v"(g));
      pr[slot] = ldg(a.rho, g);
      pt[slot] = ldg(a.th, g);
      pq[slot] = ldg(a.q, g);
      pu[slot] = ldg(uw, g);
      pe[slot] = ldg(a.u, g);
      pv[slot] = ldg(vs, g);
      pn[slot] = ldg(a.v, g);
    };
    // WIDE: this lane's chunk of the wave's two loads per level (field f,
    // 16-byte chunk c of the row segment starting at column i0-2): fields
    // 0-5 are rho, theta, q, u, v and v of row j-1; lanes 38-63 of the second
    // load repeat lane 37's chunk
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    f32x4 wa[WIDE ? PF : 1], wb[WIDE ? PF : 1];
    const float *pa = nullptr, *pb = nullptr;
    int wa_o = 0, wb_o = 0;
    float *slot_w = s_w[ty];
    const int xr = ic - i0;
    if (WIDE) {
      const int fa = tx < 51 ? tx / 17 : 3, ca = tx < 51 ? tx % 17 : tx - 51;
      const int fb = tx < 4 ? 3 : (tx < 21 ? 4 : 5);
      const int cb = tx < 4 ? 13 + tx : (tx < 21 ? tx - 4 : (tx < 38 ? tx - 21 : 16));
      const unsigned row = a.g.origin - 2u + unsigned(i0) + unsigned(j) * sj;   // column i0-2: 16-byte aligned
      auto base = [&](int f, int c) -> const float * {
        const float *fp = f == 0 ? a.rho : f == 1 ? a.th : f == 2 ? a.q : f == 3 ? a.u : a.v;
        return fp + row + unsigned(4 * c) - (f == 5 ? sj : 0u);
      };
      pa = base(fa, ca);
      pb = base(fb, cb);
      wa_o = fa * WROW + 4 * ca;
      wb_o = fb * WROW + 4 * cb;
    }
    auto fetch_w = [&](int lev, int slot) {
      size_t off = size_t(lev) * sk;
      asm volatile("" : "+v"(off));
      wa[slot] = *reinterpret_cast<const f32x4 *>(pa + off);
      wb[slot] = *reinterpret_cast<const f32x4 *>(pb + off);
    };
    // level values of this lane's column from a staged pair of loads
    auto stage_w = [&](int slot, float &r, float &t, float &q, float &ub, float &vb) {
      *reinterpret_cast<f32x4 *>(slot_w + wa_o) = wa[slot];
      *reinterpret_cast<f32x4 *>(slot_w + wb_o) = wb[slot];
      r = slot_w[xr + 2];
      t = slot_w[WROW + xr + 2];
      q = slot_w[2 * WROW + xr + 2];
      ub = (slot_w[3 * WROW + xr + 1] + slot_w[3 * WROW + xr + 2]) * 0.5f;
      vb = (slot_w[5 * WROW + xr + 2] + slot_w[4 * WROW + xr + 2]) * 0.5f;
    };
    float r0, t0, q0, ub0, vb0;
    if (WIDE) {
      // level 0 goes through slot 0 first; level PF refills it after
      fetch_w(0, 0);
#pragma unroll
      for (int l = 1; l < PF; ++l)
        if (l < NZ) fetch_w(l, l);
      stage_w(0, r0, t0, q0, ub0, vb0);
      if (PF < NZ) fetch_w(PF, 0);
    } else {
      r0 = ldg(a.rho, g0);
      t0 = ldg(a.th, g0);
      q0 = ldg(a.q, g0);
      ub0 = (ldg(uw, g0) + ldg(a.u, g0)) * 0.5f;
      vb0 = (ldg(vs, g0) + ldg(a.v, g0)) * 0.5f;
#pragma unroll
      for (int l = 1; l <= PF; ++l)
        if (l < NZ) fetch_up(l, l % PF);
    }
    const float beta = dt * r0 * ldg(a.ch, unsigned(col));
    const float ths = ldg(a.th_s, unsigned(col)), qs = ldg(a.q_s, unsigned(col));
    float dtr[NZ], dqr[NZ];
    float colr[KEEP ? NZ : 1], colt[KEEP ? NZ : 1], colq[KEEP ? NZ : 1];   // the column itself (KEEP)
    float alo = 0.f, tm1 = t0, qm1 = q0, cpv = 0.f, dtp = 0.f, dqp = 0.f, rmax = 0.f;
#pragma unroll
    for (int k = 0; k < NZ; ++k) {
      float ahi = 0.f, r1 = 0.f, t1 = t0, q1 = q0, ub1 = 0.f, vb1 = 0.f;
      if (k + 1 < NZ) {
        const int sl = (k + 1) % PF;
        if (WIDE) {
          stage_w(sl, r1, t1, q1, ub1, vb1);
          if (k + 1 + PF < NZ) fetch_w(k + 1 + PF, sl);
        } else {
          r1 = pr[sl];
          t1 = pt[sl];
          q1 = pq[sl];
          ub1 = (pu[sl] + pe[sl]) * 0.5f;
          vb1 = (pv[sl] + pn[sl]) * 0.5f;
          if (k + 1 + PF < NZ) fetch_up(k + 1 + PF, sl);
        }
        const float rdzi = s_rdzi[k];
        const float du = ub1 - ub0, dv = vb1 - vb0;
        const float kz = kmin + l2 * (__builtin_amdgcn_sqrtf(du * du + dv * dv) * rdzi);
        ahi = dt * ((r0 + r1) * 0.5f) * kz * rdzi;
      }
      if (KEEP) {
        colr[k] = r0;
        colt[k] = t0;
        colq[k] = q0;
      }
      const float m = r0 * s_dz[k];
      float diag = m + alo + ahi;
      float rt = ahi * (t1 - t0) - alo * (t0 - tm1);
      float rq = ahi * (q1 - q0) - alo * (q0 - qm1);
      if (k == 0) {
        diag += beta;
        rt += beta * (ths - t0);
        rq += beta * (qs - q0);
      }
      const float rk = (alo + ahi) * fast_rcp(m);
      rmax = rk > rmax ? rk : rmax;
      const float inv = fast_rcp(diag + alo * cpv);
      cpv = -ahi * inv;
      dtp = (rt + alo * dtp) * inv;
      dqp = (rq + alo * dqp) * inv;
      s_c[k * 256 + tid] = cpv;
      dtr[k] = dtp;
      dqr[k] = dqp;
      alo = ahi;
      tm1 = t0; t0 = t1;
      qm1 = q0; q0 = q1;
      r0 = r1; ub0 = ub1; vb0 = vb1;
      __builtin_amdgcn_sched_barrier(0);
    }

    const Column<float> c{a, g0, col, col};
    if (rmax > a.tdd) {
      const unsigned ncol = unsigned(a.g.nx) * unsigned(a.g.ny);
      const GlobalStore<double> gs{a.scratch, NZ, ncol, unsigned(col)};
      upward<float, double, 0>(c, gs);
      downward<float, double, 0, MODE>(c, gs, mass, cnt);
      fp64 = 1;
    } else {
      // ---- downward pass: back substitution, radiation suffix scan, update
      const int nx = a.g.nx, ny = a.g.ny;
      const float f0 = ldg(a.f0, unsigned(col));
      const float kappa = a.kappa, cpa = a.cp;
      const int di = ic < 2 ? nx : (ic >= nx - 2 ? -nx : 0);
      const int dj = j < 2 ? ny * int(sj) : (j >= ny - 2 ? -ny * int(sj) : 0);
      // the column's rho, theta, q come from registers (kept by the upward
      // pass; the 512-register budget of a lone wave holds them), so this
      // pass reads nothing from HBM
      const unsigned gd = g0;
      float dtn = 0.f, dqn = 0.f, tau = 0.f, tr_hi = 1.f;
      // the column's 58 mass terms are summed in plain FP64 (relative error
      // at most 57 ulp) and enter the compensated sums once per column
      double cm = 0.0, cmt = 0.0, cmq = 0.0;
      // KEEP = false: ring of the next PF levels below (slot of level k is (NZ-1-k) % PF)
      float dr[KEEP ? 1 : PF], dtt[KEEP ? 1 : PF], dqq_[KEEP ? 1 : PF];
      if (!KEEP) {
#pragma unroll
        for (int l = 0; l < PF; ++l)
          if (NZ - 1 - l >= 0) {
            unsigned g = gd + unsigned(NZ - 1 - l) * sk;
            asm volatile("" : "+v"(g));
            dr[l] = ldg(a.rho, g);
            dtt[l] = ldg(a.th, g);
            dqq_[l] = ldg(a.q, g);
          }
      }
#pragma unroll
      for (int k = NZ - 1; k >= 0; --k) {
        float r, t, q;
        if (KEEP) {
          r = colr[k];
          t = colt[k];
          q = colq[k];
        } else {
          const int sl = (NZ - 1 - k) % PF;
          r = dr[sl];
          t = dtt[sl];
          q = dqq_[sl];
          if (k - PF >= 0) {
            unsigned g = gd + unsigned(k - PF) * sk;
            asm volatile("" : "+v"(g));
            dr[sl] = ldg(a.rho, g);
            dtt[sl] = ldg(a.th, g);
            dqq_[sl] = ldg(a.q, g);
          }
        }
        const float ck = s_c[k * 256 + tid];
        const float dth = dtr[k] - ck * dtn;
        const float dqq = dqr[k] - ck * dqn;
        dtn = dth;
        dqn = dqq;
        const float dzk = s_dz[k];
        tau += kappa * r * (q > 0.f ? q : 0.f) * dzk;
        const float tr_lo = expf(-tau);
        const float heat = f0 * (tr_hi - tr_lo) * fast_rcp(cpa * (r * dzk));
        tr_hi = tr_lo;
        unsigned g = gd + unsigned(k) * sk;
        asm volatile("" : "+v"(g));
        if (MODE == 1) {
          if (a.tend_rows) {
            const unsigned o = unsigned(col) * TEND_ROW + unsigned(k);
            stg(a.tend_t, o, dth / dt + heat);
            stg(a.tend_t, o + unsigned(NZ), dqq / dt);
            if (k == 0)
              for (int p = 2 * NZ; p < TEND_ROW; ++p) stg(a.tend_t, unsigned(col) * TEND_ROW + unsigned(p), 0.f);
          } else {
            const unsigned o = unsigned(k * ny + j) * unsigned(nx) + unsigned(ic);
            stg(a.tend_t, o, dth / dt + heat);
            stg(a.tend_q, o, dqq / dt);
          }
        } else {
          const float tn = t + dth + dt * heat;
          const float qn = q + dqq;
          stg(a.th, g, tn);
          stg(a.q, g, qn);
          // (the periodic images are written after the loop: a per-lane
          // branch inside the unrolled loop keeps many more registers live)
          cnt.nonfinite += (isfinite(r) && isfinite(tn) && isfinite(qn)) ? 0 : 1;
          cnt.rho_le0 += (r > 0.f) ? 0 : 1;
          if (a.do_mass) {
            const double mv = double(r) * s_vol[k];
            cm += mv;
            cmt += mv * (double(tn) + a.theta_off);
            cmq += mv * double(qn);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      if (MODE == 0 && a.do_mass) {
        mass[0].add(cm);
        mass[1].add(cmt);
        mass[2].add(cmq);
      }
      // periodic images of the updated column (the thread reads back its own
      // stores: same addresses, program order)
      if (MODE == 0 && (di != 0 || dj != 0)) {
        for (int k = 0; k < NZ; ++k) {
          const unsigned g = gd + unsigned(k) * sk;
          const float tn = ldg(a.th, g), qn = ldg(a.q, g);
          if (di != 0) { stg(a.th, g + di, tn); stg(a.q, g + di, qn); }
          if (dj != 0) {
            stg(a.th, g + dj, tn); stg(a.q, g + dj, qn);
            if (di != 0) { stg(a.th, g + dj + di, tn); stg(a.q, g + dj + di, qn); }
          }
        }
      }
    }
  }
  if (WIDE && !active) {   // a duplicate of column nx-1 (or a row past the grid) counts nothing
    mass[0] = mass[1] = mass[2] = Kahan{};
    cnt = Counters{};
    fp64 = 0;
  }
  block_finish<4>(&a, a.partials, a.flags, MODE == 0 && a.do_mass, MODE == 0, mass, cnt, fp64);
}

// FP32 state, two lanes per column (nz even): the column physics with the
// tridiagonal solve split at mid-column (a two-sided elimination).  Lane x of
// a wave (x < 32) takes levels 0 .. H-1 of column i0 + x and eliminates
// upward from the ground, lane x + 32 takes levels H .. NZ-1 of the same
// column and eliminates downward from the lid, each with the same recurrence
// in its own march direction (its "lower" neighbour is the level it came
// from).  Their last rows meet in a 2 x 2 system for levels H-1 and H, which
// both lanes solve with the same arithmetic; each then back-substitutes
// outward.  Every diffusion coefficient (one per interface) is formed from
// the same operands as in the thread-per-column kernel.  The optical depth
// runs from the lid down: the upper lane forms it, and its heating, while it
// eliminates; the lower lane starts from the upper lane's total and forms it
// while it back-substitutes.  A lane holds half a column (c', rho and most
// of q in LDS, d', theta and the rest of q in registers), so two waves share
// each SIMD and each dependent chain is half as long as the
// thread-per-column kernel's.  32 x 4 columns
// per block; a lane past the grid edge works on column nx-1 (same values,
// same stores) and counts nothing.  Columns whose dominance ratio exceeds
// T_dd are solved whole in FP64 by their lower lane.  With a column list
// (tendency rows, MODE 1) block b takes list slots 128 b .. 128 b + 127, slot
// s writing row s; a slot past the list's length works on column 0 and
// stores nothing.
template <int NZ, int MODE>
__global__ __launch_bounds__(256, 2) void k_physics_f32_split(PhysArgs<float> a) {
  static_assert(NZ % 2 == 0, "the two halves need an even level count");
  constexpr int H = NZ / 2;
  constexpr int PF = 4;                   // levels prefetched ahead
  constexpr int QL = PHYS_SPLIT_QL < H ? PHYS_SPLIT_QL : H;   // levels of q kept in LDS
  // LDS per lane and level: c', rho, and q of the first QL levels (the rest
  // of q, d', and theta stay in registers); two blocks fit on a CU
  extern __shared__ float s_c[];          // [H][256] c', [H][256] rho, [QL][256] q
  float *s_r = s_c + H * 256, *s_q = s_c + 2 * H * 256;
  __shared__ float s_dz[NZ], s_rdzi[NZ];
  __shared__ double s_vol[NZ];
  if (a.run_if && *a.run_if == 0) return;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * 64 + tx;
  for (int k = tid; k < NZ; k += 256) {
    s_dz[k] = a.dz[k];
    s_rdzi[k] = k + 1 < NZ ? a.rdzi[k] : 0.f;
    s_vol[k] = a.vol[k];
  }
  __syncthreads();
  const int nx = a.g.nx, ny = a.g.ny;
  const bool listed = MODE == 1 && a.col_list != nullptr;
  int i, j, slot = 0;
  bool active;
  if (listed) {
    slot = blockIdx.x * 128 + ty * 32 + (tx & 31);
    active = slot < min(*a.n_list, a.list_cap);
    const int cc = active ? a.col_list[slot] : 0;
    i = cc % nx;
    j = cc / nx;
  } else {
    const int nbx = (nx + 31) / 32;
    const int L = a.reverse ? xcd_remap_rev(blockIdx.x, gridDim.x) : xcd_remap(blockIdx.x, gridDim.x);
    i = (L % nbx) * 32 + (tx & 31);
    j = (L / nbx) * 4 + ty;
    active = (i < nx) && (j < ny);
  }
  const bool up = tx >= 32;               // the upper half of the column
  const bool stores = !listed || active;  // a spare list slot computes but stores nothing
  const int ic = min(i, nx - 1);
  Kahan mass[3];
  Counters cnt;
  int fp64 = 0;
  if (j < ny) {                           // whole waves
    const unsigned sj = a.g.sj, sk = a.g.sk;
    const unsigned g0 = a.g.origin + unsigned(ic) + unsigned(j) * sj;
    const int col = ic + nx * j;
    const int trow = listed ? slot : col;   // tendency row
    const float dt = a.dt, kmin = a.kmin, l2 = a.l2, kappa = a.kappa, cpa = a.cp;
    // level and offset of local step l (0 at the ground or the lid)
    auto lev = [&](int l) { return up ? NZ - 1 - l : l; };
    const unsigned gb = up ? g0 + unsigned(NZ - 1) * sk : g0;
    auto off = [&](int l) {
      unsigned g = up ? gb - unsigned(l) * sk : gb + unsigned(l) * sk;
      asm volatile("" : "+v"(g));
      return g;
    };
    const float *uw = plane(a.u, -1), *vs = plane(a.v, -(long long)sj);
    float pr[PF], pt[PF], pq[PF], pu[PF], pe[PF], pv[PF], pn[PF];   // prefetch ring, steps l+1 .. l+PF
    auto fetch = [&](int l, int slot) {
      const unsigned g = off(l);
      pr[slot] = ldg(a.rho, g);
      pt[slot] = ldg(a.th, g);
      pq[slot] = ldg(a.q, g);
      pu[slot] = ldg(uw, g);
      pe[slot] = ldg(a.u, g);
      pv[slot] = ldg(vs, g);
      pn[slot] = ldg(a.v, g);
    };
    float r0, t0, q0, ub0, vb0;
    {
      const unsigned g = off(0);
      r0 = ldg(a.rho, g);
      t0 = ldg(a.th, g);
      q0 = ldg(a.q, g);
      ub0 = (ldg(uw, g) + ldg(a.u, g)) * 0.5f;
      vb0 = (ldg(vs, g) + ldg(a.v, g)) * 0.5f;
    }
#pragma unroll
    for (int l = 1; l <= PF; ++l)
      if (l <= H) fetch(l, l % PF);       // step H is the other half's first level
    const float beta = up ? 0.f : dt * r0 * ldg(a.ch, unsigned(col));
    const float ths = ldg(a.th_s, unsigned(col)), qs = ldg(a.q_s, unsigned(col));
    const float f0 = ldg(a.f0, unsigned(col));
    float dtr[H], dqr[H], colt[H], colq[H];
    float alo = 0.f, tm1 = t0, qm1 = q0, cpv = 0.f, dtp = 0.f, dqp = 0.f, rmax = 0.f;
    float tau1 = 0.f, trh1 = 1.f;         // optical depth from the lid (valid in the upper lane)

    // ---- first pass: toward mid-column
#pragma unroll
    for (int l = 0; l < H; ++l) {
      const int k = lev(l);
      const int sl = (l + 1) % PF;
      const float r1 = pr[sl], t1 = pt[sl], q1 = pq[sl];
      const float ub1 = (pu[sl] + pe[sl]) * 0.5f, vb1 = (pv[sl] + pn[sl]) * 0.5f;
      if (l + 1 + PF <= H) fetch(l + 1 + PF, sl);
      // the interface toward the next level of the march (k+1/2 going up, k-1/2 going down)
      const float rdzi = s_rdzi[up ? NZ - 2 - l : l];
      const float du = ub1 - ub0, dv = vb1 - vb0;
      const float kz = kmin + l2 * (__builtin_amdgcn_sqrtf(du * du + dv * dv) * rdzi);
      const float ahi = dt * ((r0 + r1) * 0.5f) * kz * rdzi;
      const float dzk = s_dz[k];
      // optical depth and heating from the lid down (the upper lane's levels)
      tau1 += kappa * r0 * (q0 > 0.f ? q0 : 0.f) * dzk;
      const float trl = expf(-tau1);
      const float heat1 = f0 * (trh1 - trl) * fast_rcp(cpa * (r0 * dzk));
      trh1 = trl;
      s_r[l * 256 + tid] = r0;
      if (l < QL) s_q[l * 256 + tid] = q0;
      else colq[l] = q0;
      {
        // the upper lane's heating enters theta (or the tendency) here; the
        // value is formed here (empty asm), not where it is used
        float ct = MODE == 0 ? (up ? t0 + dt * heat1 : t0) : (up ? heat1 : 0.f);
        asm volatile("" : "+v"(ct));
        colt[l] = ct;
      }
      const float m = r0 * dzk;
      float diag = m + alo + ahi;
      float rt = ahi * (t1 - t0) - alo * (t0 - tm1);
      float rq = ahi * (q1 - q0) - alo * (q0 - qm1);
      if (l == 0) {                         // the ground row (lower lane) takes the surface exchange
        diag += beta;
        rt += beta * (ths - t0);
        rq += beta * (qs - q0);
      }
      const float rk = (alo + ahi) * fast_rcp(m);
      rmax = rk > rmax ? rk : rmax;
      const float inv = fast_rcp(diag + alo * cpv);
      cpv = -ahi * inv;
      dtp = (rt + alo * dtp) * inv;
      dqp = (rq + alo * dqp) * inv;
      s_c[l * 256 + tid] = cpv;
      dtr[l] = dtp;
      dqr[l] = dqp;
      alo = ahi;
      tm1 = t0; t0 = t1;
      qm1 = q0; q0 = q1;
      r0 = r1; ub0 = ub1; vb0 = vb1;
      __builtin_amdgcn_sched_barrier(0);
    }

    // ---- the two halves meet: x_lo = (d_lo - c_lo d_hi) / (1 - c_lo c_hi), x_hi = d_hi - c_hi x_lo
    const float o_c = __shfl_xor(cpv, 32), o_t = __shfl_xor(dtp, 32), o_q = __shfl_xor(dqp, 32);
    const float o_rmax = __shfl_xor(rmax, 32), o_tau = __shfl_xor(tau1, 32), o_trh = __shfl_xor(trh1, 32);
    const float c_lo = up ? o_c : cpv, c_hi = up ? cpv : o_c;
    const float t_lo = up ? o_t : dtp, t_hi = up ? dtp : o_t;
    const float q_lo = up ? o_q : dqp, q_hi = up ? dqp : o_q;
    const float rden = fast_rcp(1.f - c_lo * c_hi);
    const float xt_lo = (t_lo - c_lo * t_hi) * rden, xq_lo = (q_lo - c_lo * q_hi) * rden;
    const float xt_hi = t_hi - c_hi * xt_lo, xq_hi = q_hi - c_hi * xq_lo;
    const float rcol = rmax > o_rmax ? rmax : o_rmax;

    if (rcol > a.tdd) {
      if (!up && stores) {
        const Column<float> c{a, g0, col, trow};
        const unsigned ncol = unsigned(nx) * unsigned(ny);
        const GlobalStore<double> gs{a.scratch, NZ, ncol, unsigned(col)};
        upward<float, double, 0>(c, gs);
        downward<float, double, 0, MODE>(c, gs, mass, cnt);
        fp64 = 1;
      }
    } else {
      // ---- second pass: back substitution outward, the lower lane's optical depth, update
      const int di = ic < 2 ? nx : (ic >= nx - 2 ? -nx : 0);
      const int dj = j < 2 ? ny * int(sj) : (j >= ny - 2 ? -ny * int(sj) : 0);
      // the first unknown past this half's last row: level H for the lower lane, H-1 for the upper
      float dtn = up ? xt_lo : xt_hi, dqn = up ? xq_lo : xq_hi;
      float tau2 = o_tau, trh2 = o_trh;       // the lower lane continues the upper lane's optical depth
      double cm = 0.0, cmt = 0.0, cmq = 0.0;
#pragma unroll
      for (int l = H - 1; l >= 0; --l) {
        const int k = lev(l);
        const float ck = s_c[l * 256 + tid];
        const float dth = dtr[l] - ck * dtn;
        const float dqq = dqr[l] - ck * dqn;
        dtn = dth;
        dqn = dqq;
        const float r = s_r[l * 256 + tid], q = l < QL ? s_q[l * 256 + tid] : colq[l], dzk = s_dz[k];
        tau2 += kappa * r * (q > 0.f ? q : 0.f) * dzk;
        const float trl = expf(-tau2);
        const float heat2 = up ? 0.f : f0 * (trh2 - trl) * fast_rcp(cpa * (r * dzk));
        trh2 = trl;
        const unsigned g = off(l);
        if (MODE == 1) {
          const float heat = colt[l] + heat2;
          if (a.tend_rows) {
            const unsigned o = unsigned(trow) * TEND_ROW + unsigned(k);
            if (stores) {
              stg(a.tend_t, o, dth / dt + heat);
              stg(a.tend_t, o + unsigned(NZ), dqq / dt);
            }
          } else {
            const unsigned o = unsigned(k * ny + j) * unsigned(nx) + unsigned(ic);
            stg(a.tend_t, o, dth / dt + heat);
            stg(a.tend_q, o, dqq / dt);
          }
        } else {
          const float tn = colt[l] + dth + dt * heat2;
          const float qn = q + dqq;
          stg(a.th, g, tn);
          stg(a.q, g, qn);
          cnt.nonfinite += (isfinite(r) && isfinite(tn) && isfinite(qn)) ? 0 : 1;
          cnt.rho_le0 += (r > 0.f) ? 0 : 1;
          if (a.do_mass) {
            const double mv = double(r) * s_vol[k];
            cm += mv;
            cmt += mv * (double(tn) + a.theta_off);
            cmq += mv * double(qn);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      if (MODE == 1 && a.tend_rows && !up && stores)
        for (int p = 2 * NZ; p < TEND_ROW; ++p) stg(a.tend_t, unsigned(trow) * TEND_ROW + unsigned(p), 0.f);
      if (MODE == 0 && a.do_mass) {
        mass[0].add(cm);
        mass[1].add(cmt);
        mass[2].add(cmq);
      }
      // periodic images of this half's levels (the lane reads back its own stores)
      if (MODE == 0 && (di != 0 || dj != 0)) {
        for (int l = 0; l < H; ++l) {
          const unsigned g = off(l);
          const float tn = ldg(a.th, g), qn = ldg(a.q, g);
          if (di != 0) { stg(a.th, g + di, tn); stg(a.q, g + di, qn); }
          if (dj != 0) {
            stg(a.th, g + dj, tn); stg(a.q, g + dj, qn);
            if (di != 0) { stg(a.th, g + dj + di, tn); stg(a.q, g + dj + di, qn); }
          }
        }
      }
    }
  }
  if (!active) {   // a duplicate of column nx-1 (or a row past the grid) counts nothing
    mass[0] = mass[1] = mass[2] = Kahan{};
    cnt = Counters{};
    fp64 = 0;
  }
  block_finish<4>(&a, a.partials, a.flags, MODE == 0 && a.do_mass, MODE == 0, mass, cnt, fp64);
}

template <typename T, int MODE>
__global__ __launch_bounds__(PHYS_BX) void k_physics(PhysArgs<T> a) {
  extern __shared__ unsigned char s_raw[];
  if (a.run_if && *a.run_if == 0) return;
  const int lane = threadIdx.x;
  int i, j, row;
  bool active;
  if (a.col_list) {                       // listed columns (tendency rows by slot)
    row = blockIdx.x * PHYS_BX + lane;
    active = row < min(*a.n_list, a.list_cap);
    const int cc = active ? a.col_list[row] : 0;
    i = cc % a.g.nx;
    j = cc / a.g.nx;
  } else {
    const int nbx = (a.g.nx + PHYS_BX - 1) / PHYS_BX;
    j = blockIdx.x / nbx;
    i = (blockIdx.x % nbx) * PHYS_BX + lane;
    active = i < a.g.nx;
    row = i + a.g.nx * j;
  }
  Kahan mass[3];
  Counters cnt;
  int fp64 = 0;
  if (active) {
    const Column<T> c{a, a.g.origin + unsigned(i) + unsigned(j) * a.g.sj, i + a.g.nx * j, row};
    const unsigned ncol = unsigned(a.g.nx) * unsigned(a.g.ny);
    bool wide;
    if (sizeof(T) == 4) {
      if (a.use_lds) {
        const LdsStore<float> st{reinterpret_cast<float *>(s_raw), a.g.nz, lane};
        wide = upward<T, float, 0>(c, st) > a.tdd;
        if (!wide) downward<T, float, 0, MODE>(c, st, mass, cnt);
      } else {
        const GlobalStore<float> st{reinterpret_cast<float *>(a.scratch), a.g.nz, ncol, unsigned(c.col)};
        wide = upward<T, float, 0>(c, st) > a.tdd;
        if (!wide) downward<T, float, 0, MODE>(c, st, mass, cnt);
      }
    } else {
      const GlobalStore<double> st{a.scratch, a.g.nz, ncol, unsigned(c.col)};
      wide = upward<T, double, 0>(c, st) > a.tdd;
      downward<T, double, 0, MODE>(c, st, mass, cnt);
      fp64 = wide ? 1 : 0;
      wide = false;
    }
    if (wide) {
      const GlobalStore<double> st{a.scratch, a.g.nz, ncol, unsigned(c.col)};
      upward<T, double, 0>(c, st);
      downward<T, double, 0, MODE>(c, st, mass, cnt);
      fp64 = 1;
    }
  }
  // block (= one wave) reductions in a fixed order
  const int nf = wave_sum_int(cnt.nonfinite), nr = wave_sum_int(cnt.rho_le0), nd = wave_sum_int(fp64);
  if (MODE == 0 && a.do_mass) {
    for (int v = 0; v < 3; ++v) wave_merge(mass[v]);
    if (lane == 0) {
      double *p = a.partials + (long long)blockIdx.x * 6;
      for (int v = 0; v < 3; ++v) {
        p[2 * v] = mass[v].s;
        p[2 * v + 1] = mass[v].c;
      }
    }
  }
  if (lane == 0 && MODE == 0) {
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
    const unsigned g0 = a.g.origin + unsigned(i) + unsigned(j) * a.g.sj;
    for (int k = 0; k < a.g.nz; ++k) {
      const unsigned g = g0 + unsigned(k) * a.g.sk;
      const T r = ldg(a.rho, g), t = ldg(a.th, g), q = ldg(a.q, g);
      if (!(isfinite(r) && isfinite(t) && isfinite(q))) cnt.nonfinite++;
      if (!(r > T(0))) cnt.rho_le0++;
      const double mv = double(r) * a.vol[k];
      mass[0].add(mv);
      mass[1].add(mv * (double(t) + a.theta_off));
      mass[2].add(mv * double(q));
    }
  }
  for (int v = 0; v < 3; ++v) wave_merge(mass[v]);
  const int nf = wave_sum_int(cnt.nonfinite), nr = wave_sum_int(cnt.rho_le0);
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
  if (a.col_list) {
    if (a.mode != 1 || a.list_cap <= 0) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 4) {
      // listed tendency rows of 58-level columns: the two-lane kernel
      if (a.variant == PHYS_VARIANT_SPLIT && a.tend_rows && a.g.nz == 58) {
        hipLaunchKernelGGL((k_physics_f32_split<58, 1>), dim3((a.list_cap + 127) / 128), dim3(64, 4),
                           phys_split_lds(58), s, a);
        return hipGetLastError();
      }
    }
    const int nb = (a.list_cap + PHYS_BX - 1) / PHYS_BX;
    const size_t lds = (sizeof(T) == 4 && a.use_lds) ? size_t(3) * a.g.nz * PHYS_BX * sizeof(float) : 0;
    hipLaunchKernelGGL((k_physics<T, 1>), dim3(nb), dim3(PHYS_BX), lds, s, a);
    return hipGetLastError();
  }
  if constexpr (sizeof(T) == 4) {
    if (phys_uses_scan(4, a.g.nz, a.variant) && !a.tend_rows) return launch_physics_scan(a, s);
    const int nb = phys_reg_blocks(a.g.nx, a.g.ny);
    const dim3 blk(64, 4);
    if (a.variant == PHYS_VARIANT_SPLIT && (a.g.nz == 58 || a.g.nz == 16)) {
      const int nbs = phys_split_blocks(a.g.nx, a.g.ny);
      const size_t lds = phys_split_lds(a.g.nz);
      if (a.g.nz == 58) {
        if (a.mode == 0) hipLaunchKernelGGL((k_physics_f32_split<58, 0>), dim3(nbs), blk, lds, s, a);
        else hipLaunchKernelGGL((k_physics_f32_split<58, 1>), dim3(nbs), blk, lds, s, a);
      } else {
        if (a.mode == 0) hipLaunchKernelGGL((k_physics_f32_split<16, 0>), dim3(nbs), blk, lds, s, a);
        else hipLaunchKernelGGL((k_physics_f32_split<16, 1>), dim3(nbs), blk, lds, s, a);
      }
      return hipGetLastError();
    }
    const bool keep = a.variant != PHYS_VARIANT_REREAD;
    const bool wide = a.variant == PHYS_VARIANT_WIDE;
    if (a.g.nz == 58) {
      const size_t lds = 58 * 256 * sizeof(float);
      if (wide) {
        if (a.mode == 0) hipLaunchKernelGGL((k_physics_f32<58, 0, true, true>), dim3(nb), blk, lds, s, a);
        else hipLaunchKernelGGL((k_physics_f32<58, 1, true, true>), dim3(nb), blk, lds, s, a);
      } else if (keep) {
        if (a.mode == 0) hipLaunchKernelGGL((k_physics_f32<58, 0, true>), dim3(nb), blk, lds, s, a);
        else hipLaunchKernelGGL((k_physics_f32<58, 1, true>), dim3(nb), blk, lds, s, a);
      } else {
        if (a.mode == 0) hipLaunchKernelGGL((k_physics_f32<58, 0, false>), dim3(nb), blk, lds, s, a);
        else hipLaunchKernelGGL((k_physics_f32<58, 1, false>), dim3(nb), blk, lds, s, a);
      }
      return hipGetLastError();
    }
    if (a.g.nz == 16) {
      const size_t lds = 16 * 256 * sizeof(float);
      if (wide) {
        if (a.mode == 0) hipLaunchKernelGGL((k_physics_f32<16, 0, true, true>), dim3(nb), blk, lds, s, a);
        else hipLaunchKernelGGL((k_physics_f32<16, 1, true, true>), dim3(nb), blk, lds, s, a);
      } else if (keep) {
        if (a.mode == 0) hipLaunchKernelGGL((k_physics_f32<16, 0, true>), dim3(nb), blk, lds, s, a);
        else hipLaunchKernelGGL((k_physics_f32<16, 1, true>), dim3(nb), blk, lds, s, a);
      } else {
        if (a.mode == 0) hipLaunchKernelGGL((k_physics_f32<16, 0, false>), dim3(nb), blk, lds, s, a);
        else hipLaunchKernelGGL((k_physics_f32<16, 1, false>), dim3(nb), blk, lds, s, a);
      }
      return hipGetLastError();
    }
  }
  const int nb = phys_blocks(a.g.nx, a.g.ny);
  const size_t lds = (sizeof(T) == 4 && a.use_lds) ? size_t(3) * a.g.nz * PHYS_BX * sizeof(float) : 0;
  if (a.mode == 0) hipLaunchKernelGGL((k_physics<T, 0>), dim3(nb), dim3(PHYS_BX), lds, s, a);
  else hipLaunchKernelGGL((k_physics<T, 1>), dim3(nb), dim3(PHYS_BX), lds, s, a);
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
