// HEVI fast-mode short step: the linear acoustic-gravity system integrated
// horizontally explicit, vertically implicit (section "The ASUCA Weather
// Prediction Model": sound and gravity waves are split from the Runge-Kutta
// long step and advanced in shorter steps of a second-order Runge-Kutta
// scheme, HEVI; section "Hybrid ASUCA Strong Scaling GPU Results" names
// these fast modes as the costliest module).  The equations are readings:
//   du/dt = -dpi/dx, dv/dt = -dpi/dy, dw/dt = -dpi/dz + b, db/dt = -N^2 w,
//   dpi/dt = -c^2 div(u, v, w)
// on the C-grid of the dycore (u east faces, v north faces, pi cells, w and b
// on the nz + 1 level faces, w = b = 0 at ground and lid).  A short step of
// length tau is two stages from the step's base state X, h = tau/2 then tau,
// each using the previous stage's pi horizontally:
//   u' = u - h dpi_prev/dx,  v' = v - h dpi_prev/dy,  D = du'/dx + dv'/dy,
//   (1 + h^2 N^2/4) wm - (h^2 c^2/4) d/dz(dwm/dz)
//        = w + (h/2)(-dpi/dz + b) + (h^2 c^2/4) dD/dz      (interior faces)
//   w' = 2 wm - w,  b' = b - h N^2 wm,  pi' = pi - h c^2 (D + dwm/dz).
//
// GPU design: one thread per column, 64 x 4 columns per block (i coalesced),
// k marched twice like the column physics.  The tridiagonal matrix is the
// same in every column (it depends on dz, h, c, N only), so its Thomas
// factors are computed once on the host and read from a small table; a
// column only carries its right-hand side through the forward sweep.  The
// upward march forms D and the right-hand side level by level from a
// one-level look-behind in registers and parks D in the pi output and the
// eliminated right-hand side in the w output (or a scratch face field),
// both re-read by the same thread on the way down, where the back
// substitution yields wm and the final w', b', pi'.  The first stage only
// needs pi' (the second stage starts again from X), so it writes nothing
// else.  Outputs write their own periodic halo images.
#include "wx_internal.h"

namespace wx {
namespace {

// x / d in FP64 (as the definition divides), x * (1/d) in FP32
__device__ __forceinline__ double over(double x, double d, double) { return x / d; }
__device__ __forceinline__ float over(float x, float, float rd) { return x * rd; }

template <typename T, bool FULL>
__global__ __launch_bounds__(256) void k_hevi_stage(HeviArgs<T> a) {
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int nbx = (nx + 63) / 64;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int i = (L % nbx) * 64 + threadIdx.x, j = (L / nbx) * 4 + threadIdx.y;
  if (i >= nx || j >= ny) return;
  const unsigned sj = a.g.sj, sk = a.g.sk;
  const unsigned col = a.g.origin + unsigned(i) + unsigned(j) * sj;
  const long long sjl = sj;
  // neighbours through shifted uniform bases: one vector offset per level
  const T *pe = plane(a.pp, 1), *pw = plane(a.pp, -1), *pn = plane(a.pp, sjl), *ps = plane(a.pp, -sjl);
  const T *uw = plane(a.u, -1), *vs = plane(a.v, -sjl);
  const T h = a.h, h2 = a.h2, a4 = a.a4, hc2 = a.hc2, hn2 = a.hn2, dx = a.dx, rdx = a.rdx;
  const HeviCoef<T> *cf = a.coef;
  const int di = i < 2 ? nx : (i >= nx - 2 ? -nx : 0);
  const int dj = j < 2 ? ny * int(sj) : (j >= ny - 2 ? -ny * int(sj) : 0);
  auto put = [&](T *f, unsigned g, T v) {
    stg(f, g, v);
    if (di != 0) stg(f, g + di, v);
    if (dj != 0) {
      stg(f, g + dj, v);
      if (di != 0) stg(f, g + dj + di, v);
    }
  };

  // ---- upward: D, the u'/v' winds, the right-hand side and its elimination
  T d_lo = 0, pi_lo = 0, e_lo = 0;
  for (int k = 0; k < nz; ++k) {
    const unsigned g = col + unsigned(k) * sk;
    const T pc = ldg(a.pp, g);
    const T ue = ldg(a.u, g) - over(h * (ldg(pe, g) - pc), dx, rdx);
    const T uo = ldg(uw, g) - over(h * (pc - ldg(pw, g)), dx, rdx);
    const T vn = ldg(a.v, g) - over(h * (ldg(pn, g) - pc), dx, rdx);
    const T vo = ldg(vs, g) - over(h * (pc - ldg(ps, g)), dx, rdx);
    const T D = over(ue - uo, dx, rdx) + over(vn - vo, dx, rdx);
    if (FULL) {
      put(a.u_o, g, ue);
      put(a.v_o, g, vn);
    }
    stg(a.pi_o, g, D);                      // parked until the way down
    const T pik = ldg(a.pi, g);
    if (k > 0) {
      const HeviCoef<T> c = cf[k];          // face f = k, between cells k-1 and k
      const T rhs = (ldg(a.w, g) + h2 * (over(-(pik - pi_lo), c.dzf, c.rdzf) + ldg(a.b, g))) +
                    over(a4 * (D - d_lo), c.dzf, c.rdzf);
      const T e = (rhs + c.lo * e_lo) * c.inv;
      stg(a.e_o, g, e);                     // parked until the way down
      e_lo = e;
    }
    d_lo = D;
    pi_lo = pik;
  }

  // ---- downward: back substitution, w', b', pi'
  T wm_hi = 0;                              // wm at the face above (the lid: 0)
  for (int k = nz - 1; k >= 0; --k) {
    const unsigned g = col + unsigned(k) * sk;
    const HeviCoef<T> c = cf[k];
    T wm = 0;                               // wm at face k (the ground: 0)
    if (k > 0) {
      wm = ldg(a.e_o, g) - c.cp * wm_hi;
      if (FULL) {
        const T wk = ldg(a.w, g);
        stg(a.w_o, g, T(2) * wm - wk);
        stg(a.b_o, g, ldg(a.b, g) - hn2 * wm);
      }
    }
    put(a.pi_o, g, ldg(a.pi, g) - hc2 * (ldg(a.pi_o, g) + over(wm_hi - wm, c.dz, c.rdz)));
    wm_hi = wm;
  }
  if (FULL) {
    const unsigned g0 = col, gt = col + unsigned(nz) * sk;
    stg(a.w_o, g0, T(0));
    stg(a.w_o, gt, T(0));
    stg(a.b_o, g0, T(0));
    stg(a.b_o, gt, T(0));
  }
}

// The same stage for a compile-time level count (the 58- and 16-level
// grids): the column's P_k = pi_k - h c^2 D_k and eliminated right-hand side
// e_f stay in registers between the two marches instead of round-tripping
// through memory, so the first stage moves exactly its five inputs and its
// pi, and the second re-reads only w and b on the way down.  P_k forms
// pi - h c^2 (D + dwm/dz) as (pi - h c^2 D) - h c^2 dwm/dz, one rounding
// more than the generic kernel.
template <typename T, bool FULL, int NZ>
__global__ __launch_bounds__(256) void k_hevi_stage_reg(HeviArgs<T> a) {
  const int nx = a.g.nx, ny = a.g.ny;
  const int nbx = (nx + 63) / 64;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int i = (L % nbx) * 64 + threadIdx.x, j = (L / nbx) * 4 + threadIdx.y;
  if (i >= nx || j >= ny) return;
  const unsigned sj = a.g.sj, sk = a.g.sk;
  const unsigned col = a.g.origin + unsigned(i) + unsigned(j) * sj;
  const long long sjl = sj;
  const T *pe = plane(a.pp, 1), *pw = plane(a.pp, -1), *pn = plane(a.pp, sjl), *ps = plane(a.pp, -sjl);
  const T *uw = plane(a.u, -1), *vs = plane(a.v, -sjl);
  const T h = a.h, h2 = a.h2, a4 = a.a4, hc2 = a.hc2, hn2 = a.hn2, dx = a.dx, rdx = a.rdx;
  const HeviCoef<T> *cf = a.coef;
  const int di = i < 2 ? nx : (i >= nx - 2 ? -nx : 0);
  const int dj = j < 2 ? ny * int(sj) : (j >= ny - 2 ? -ny * int(sj) : 0);
  T P[NZ], E[NZ];
  T d_lo = 0, pi_lo = 0, e_lo = 0;
  // the twelve loads of a level are issued PF levels ahead (a register ring)
  constexpr int PF = 3;
  T rc[PF], re[PF], rw[PF], rn[PF], rs[PF], ru[PF], rv[PF], rx[PF], ry[PF], rp[PF], rwz[PF], rbz[PF];
  auto fetch = [&](int lev, int sl) {
    // an opaque per-level offset keeps the compiler from computing every
    // level's address up front (NZ more live registers)
    unsigned g = col + unsigned(lev) * sk;
    asm volatile("" : "+v"(g));
    rc[sl] = ldg(a.pp, g);
    re[sl] = ldg(pe, g);
    rw[sl] = ldg(pw, g);
    rn[sl] = ldg(pn, g);
    rs[sl] = ldg(ps, g);
    ru[sl] = ldg(a.u, g);
    rx[sl] = ldg(uw, g);
    rv[sl] = ldg(a.v, g);
    ry[sl] = ldg(vs, g);
    rp[sl] = ldg(a.pi, g);
    rwz[sl] = ldg(a.w, g);
    rbz[sl] = ldg(a.b, g);
  };
#pragma unroll
  for (int l = 0; l < PF; ++l)
    if (l < NZ) fetch(l, l);
#pragma unroll
  for (int k = 0; k < NZ; ++k) {
    const int sl = k % PF;
    unsigned g = col + unsigned(k) * sk;
    asm volatile("" : "+v"(g));
    const T pc = rc[sl];
    const T ue = ru[sl] - over(h * (re[sl] - pc), dx, rdx);
    const T uo = rx[sl] - over(h * (pc - rw[sl]), dx, rdx);
    const T vn = rv[sl] - over(h * (rn[sl] - pc), dx, rdx);
    const T vo = ry[sl] - over(h * (pc - rs[sl]), dx, rdx);
    const T D = over(ue - uo, dx, rdx) + over(vn - vo, dx, rdx);
    if (FULL) {
      stg(a.u_o, g, ue);
      stg(a.v_o, g, vn);
    }
    const T pik = rp[sl], wk = rwz[sl], bk = rbz[sl];
    if (k + PF < NZ) fetch(k + PF, sl);
    P[k] = pik - hc2 * D;
    if (k > 0) {
      const HeviCoef<T> c = cf[k];
      const T rhs = (wk + h2 * (over(-(pik - pi_lo), c.dzf, c.rdzf) + bk)) +
                    over(a4 * (D - d_lo), c.dzf, c.rdzf);
      const T e = (rhs + c.lo * e_lo) * c.inv;
      E[k] = e;
      e_lo = e;
    }
    d_lo = D;
    pi_lo = pik;
    __builtin_amdgcn_sched_barrier(0);
  }
  // the coefficients are read again on the way down through an opaque copy
  // of the table pointer: reusing the upward march's values would keep all
  // NZ levels of them live in registers across both marches
  const HeviCoef<T> *cfd = cf;
  asm volatile("" : "+s"(cfd));
  T wm_hi = 0;
  // w and b of the second stage, re-read on the way down PF levels ahead
  T dw[PF], db[PF];
  auto fetch_dn = [&](int lev, int sl) {
    unsigned g = col + unsigned(lev) * sk;
    asm volatile("" : "+v"(g));
    dw[sl] = ldg(a.w, g);
    db[sl] = ldg(a.b, g);
  };
  if (FULL) {
#pragma unroll
    for (int l = 0; l < PF; ++l)
      if (NZ - 1 - l >= 1) fetch_dn(NZ - 1 - l, l);
  }
#pragma unroll
  for (int k = NZ - 1; k >= 0; --k) {
    unsigned g = col + unsigned(k) * sk;
    asm volatile("" : "+v"(g));
    const HeviCoef<T> c = cfd[k];
    T wm = 0;
    if (k > 0) {
      wm = E[k] - c.cp * wm_hi;
      if (FULL) {
        const int sl = (NZ - 1 - k) % PF;
        const T wk = dw[sl], bk = db[sl];
        if (k - PF >= 1) fetch_dn(k - PF, sl);
        stg(a.w_o, g, T(2) * wm - wk);
        stg(a.b_o, g, bk - hn2 * wm);
      }
    }
    stg(a.pi_o, g, P[k] - hc2 * over(wm_hi - wm, c.dz, c.rdz));
    wm_hi = wm;
    __builtin_amdgcn_sched_barrier(0);
  }
  if (FULL) {
    stg(a.w_o, col, T(0));
    stg(a.w_o, col + unsigned(NZ) * sk, T(0));
    stg(a.b_o, col, T(0));
    stg(a.b_o, col + unsigned(NZ) * sk, T(0));
  }
  // periodic halo images, written after both marches: a branch on the lane
  // inside the unrolled marches would keep far more registers live.  The
  // thread reads back its own stores (same addresses, program order).
  if (di != 0 || dj != 0) {
    for (int k = 0; k < NZ; ++k) {
      const unsigned g = col + unsigned(k) * sk;
      T *outs[3] = {a.pi_o, a.u_o, a.v_o};
      for (int f = 0; f < (FULL ? 3 : 1); ++f) {
        const T v = ldg(outs[f], g);
        if (di != 0) stg(outs[f], g + di, v);
        if (dj != 0) {
          stg(outs[f], g + dj, v);
          if (di != 0) stg(outs[f], g + dj + di, v);
        }
      }
    }
  }
}

// The register kernel's stage with two lanes per column (nz even): lane x
// of a wave (x < 32) takes cells 0 .. H-1 and faces 1 .. H-1 of column
// i0 + x, lane x + 32 cells H .. nz-1 and faces H+1 .. nz-1 of the same
// column.  The lower lane eliminates from the ground up with the usual
// factors, the upper lane from the lid down with factors eliminated in that
// direction (both from the two-sided table, coef2); face H joins them in one
// row that both lanes solve with the same operands; then each lane
// back-substitutes outward.  Every right-hand side is formed from the same
// operands as in the one-sided kernels.  Half a column per lane halves the
// registers per lane (218 at nz = 58: two waves per SIMD) and the length of each
// dependent chain.  32 x R columns per block, R = blockDim.y: 8 for the
// second stage (the neighbour rows its divergence reads from outside the
// block are an eighth of its own), 4 for the first, which reads fewer fields
// (2.46 ms per short step with 8 rows for both, 2.43 with 8 and 4, 2.54 with
// 4 and 8, 2.48 with 8 and 2); a lane past the grid edge works
// on column nx-1 (the same values and the same stores).
template <typename T, bool FULL, int NZ>
__global__ __launch_bounds__(512) void k_hevi_stage_split(HeviArgs<T> a) {
  static_assert(NZ % 2 == 0 && NZ >= 4, "two halves of at least two cells");
  constexpr int H = NZ / 2;
  // the two-sided table, staged once per block: read per lane (the halves
  // read different faces) through an opaque index per level, so that the
  // compiler forms each level's reads where they are used
  __shared__ HeviCoef<T> s_cf[NZ];
  {
    const int t = threadIdx.y * 64 + threadIdx.x;
    if (t < NZ) s_cf[t] = a.coef2[t];
  }
  __syncthreads();
  const int nx = a.g.nx, ny = a.g.ny;
  const int nbx = (nx + 31) / 32;
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int i = (L % nbx) * 32 + (int(threadIdx.x) & 31), j = (L / nbx) * int(blockDim.y) + int(threadIdx.y);
  if (j >= ny) return;                     // whole waves
  const bool up = threadIdx.x >= 32;
  const int ic = min(i, nx - 1);
  const unsigned sj = a.g.sj, sk = a.g.sk;
  const unsigned col = a.g.origin + unsigned(ic) + unsigned(j) * sj;
  const long long sjl = sj;
  const T *pe = plane(a.pp, 1), *pw = plane(a.pp, -1), *pn = plane(a.pp, sjl), *ps = plane(a.pp, -sjl);
  const T *uw = plane(a.u, -1), *vs = plane(a.v, -sjl);
  const T h = a.h, h2 = a.h2, a4 = a.a4, hc2 = a.hc2, hn2 = a.hn2, dx = a.dx, rdx = a.rdx;
  auto tab = [&](int idx) {
    asm volatile("" : "+v"(idx));
    return s_cf[idx];
  };
  const int di = ic < 2 ? nx : (ic >= nx - 2 ? -nx : 0);
  const int dj = j < 2 ? ny * int(sj) : (j >= ny - 2 ? -ny * int(sj) : 0);
  // cell and face of local step l: the lower lane climbs from cell 0 (face l
  // below cell l), the upper lane descends from cell nz-1 (face nz-l above
  // cell nz-1-l)
  auto cell = [&](int l) { return up ? NZ - 1 - l : l; };
  auto face = [&](int l) { return up ? NZ - l : l; };
  auto coff = [&](int l) {
    unsigned g = col + unsigned(cell(l)) * sk;
    asm volatile("" : "+v"(g));
    return g;
  };
  auto foff = [&](int l) {
    unsigned g = col + unsigned(face(l)) * sk;
    asm volatile("" : "+v"(g));
    return g;
  };
  T P[H], E[H];
  T d_prev = 0, pi_prev = 0, e_prev = 0;
  constexpr int PF = 3;
  T rc[PF], re[PF], rw[PF], rn[PF], rs[PF], ru[PF], rv[PF], rx[PF], ry[PF], rp[PF], rwz[PF], rbz[PF];
  auto fetch = [&](int l, int sl) {
    const unsigned g = coff(l), gf = foff(l);
    rc[sl] = ldg(a.pp, g);
    re[sl] = ldg(pe, g);
    rw[sl] = ldg(pw, g);
    rn[sl] = ldg(pn, g);
    rs[sl] = ldg(ps, g);
    ru[sl] = ldg(a.u, g);
    rx[sl] = ldg(uw, g);
    rv[sl] = ldg(a.v, g);
    ry[sl] = ldg(vs, g);
    rp[sl] = ldg(a.pi, g);
    rwz[sl] = ldg(a.w, gf);
    rbz[sl] = ldg(a.b, gf);
  };
#pragma unroll
  for (int l = 0; l < PF; ++l)
    if (l < H) fetch(l, l);
  // ---- first pass: toward face H
#pragma unroll
  for (int l = 0; l < H; ++l) {
    const int sl = l % PF;
    const unsigned g = coff(l);
    const T pc = rc[sl];
    const T ue = ru[sl] - over(h * (re[sl] - pc), dx, rdx);
    const T uo = rx[sl] - over(h * (pc - rw[sl]), dx, rdx);
    const T vn = rv[sl] - over(h * (rn[sl] - pc), dx, rdx);
    const T vo = ry[sl] - over(h * (pc - rs[sl]), dx, rdx);
    const T D = over(ue - uo, dx, rdx) + over(vn - vo, dx, rdx);
    if (FULL) {
      stg(a.u_o, g, ue);
      stg(a.v_o, g, vn);
    }
    const T pik = rp[sl], wk = rwz[sl], bk = rbz[sl];
    if (l + PF < H) fetch(l + PF, sl);
    P[l] = pik - hc2 * D;
    if (l > 0) {
      // the face between this cell and the previous one: above - below
      const HeviCoef<T> c = tab(face(l));
      const T pi_a = up ? pi_prev : pik, pi_b = up ? pik : pi_prev;
      const T d_a = up ? d_prev : D, d_b = up ? D : d_prev;
      const T rhs = (wk + h2 * (over(-(pi_a - pi_b), c.dzf, c.rdzf) + bk)) + over(a4 * (d_a - d_b), c.dzf, c.rdzf);
      const T e = (rhs + c.lo * e_prev) * c.inv;
      E[l] = e;
      e_prev = e;
    }
    d_prev = D;
    pi_prev = pik;
    __builtin_amdgcn_sched_barrier(0);
  }
  // ---- face H: the row joining the halves, solved alike in both lanes
  const T o_e = __shfl_xor(e_prev, 32), o_d = __shfl_xor(d_prev, 32), o_pi = __shfl_xor(pi_prev, 32);
  const T e_lo = up ? o_e : e_prev, e_hi = up ? e_prev : o_e;        // E_{H-1}, E'_{H+1}
  const T d_lo = up ? o_d : d_prev, d_hi = up ? d_prev : o_d;        // D of cells H-1, H
  const T pi_lo = up ? o_pi : pi_prev, pi_hi = up ? pi_prev : o_pi;  // pi of cells H-1, H
  const unsigned gH = col + unsigned(H) * sk;
  const T wH = ldg(a.w, gH), bH = ldg(a.b, gH);
  T wm_mid;
  {
    const HeviCoef<T> c = s_cf[H];
    const T rhs = (wH + h2 * (over(-(pi_hi - pi_lo), c.dzf, c.rdzf) + bH)) + over(a4 * (d_hi - d_lo), c.dzf, c.rdzf);
    wm_mid = ((rhs + c.lo * e_lo) + c.pad * e_hi) * c.inv;
  }
  if (FULL && !up) {
    stg(a.w_o, gH, T(2) * wm_mid - wH);
    stg(a.b_o, gH, bH - hn2 * wm_mid);
  }
  // ---- second pass: back substitution outward, w', b', pi'
  T dw[PF], db[PF];
  auto fetch_dn = [&](int l, int sl) {
    const unsigned gf = foff(l);
    dw[sl] = ldg(a.w, gf);
    db[sl] = ldg(a.b, gf);
  };
  if (FULL) {
#pragma unroll
    for (int q = 0; q < PF; ++q)
      if (H - 1 - q >= 1) fetch_dn(H - 1 - q, q);
  }
  T wm_prev = wm_mid;
#pragma unroll
  for (int l = H - 1; l >= 0; --l) {
    const HeviCoef<T> c = tab(cell(l));
    const unsigned g = coff(l);
    T wm = 0;                              // the ground (lower lane) or the lid (upper lane) at l = 0
    if (l > 0) {
      const HeviCoef<T> cfc = tab(face(l));
      wm = E[l] - cfc.cp * wm_prev;
      if (FULL) {
        const int sl = (H - 1 - l) % PF;
        const T wk = dw[sl], bk = db[sl];
        if (l - PF >= 1) fetch_dn(l - PF, sl);
        const unsigned gf = foff(l);
        stg(a.w_o, gf, T(2) * wm - wk);
        stg(a.b_o, gf, bk - hn2 * wm);
      }
    }
    // the cell between this face and the previous one: above - below
    const T w_a = up ? wm : wm_prev, w_b = up ? wm_prev : wm;
    stg(a.pi_o, g, P[l] - hc2 * over(w_a - w_b, c.dz, c.rdz));
    wm_prev = wm;
    __builtin_amdgcn_sched_barrier(0);
  }
  if (FULL) {
    const unsigned gb = up ? col + unsigned(NZ) * sk : col;   // lid or ground face
    stg(a.w_o, gb, T(0));
    stg(a.b_o, gb, T(0));
  }
  // periodic halo images of this half's cells (the lane reads back its own stores)
  if (di != 0 || dj != 0) {
    for (int l = 0; l < H; ++l) {
      const unsigned g = col + unsigned(cell(l)) * sk;
      T *outs[3] = {a.pi_o, a.u_o, a.v_o};
      for (int f = 0; f < (FULL ? 3 : 1); ++f) {
        const T v = ldg(outs[f], g);
        if (di != 0) stg(outs[f], g + di, v);
        if (dj != 0) {
          stg(outs[f], g + dj, v);
          if (di != 0) stg(outs[f], g + dj + di, v);
        }
      }
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_hevi_stage(const HeviArgs<T> &a, bool full, int kernel, hipStream_t s) {
  const int nb = ((a.g.nx + 63) / 64) * ((a.g.ny + 3) / 4);
  const bool fixed = a.g.nz == 58 || a.g.nz == 16;
  if (kernel == 2 && fixed) {
    // 32 x 8 columns per block for the second stage, 32 x 4 for the first
    const int rows = full ? 8 : 4;
    const int nb2 = ((a.g.nx + 31) / 32) * ((a.g.ny + rows - 1) / rows);
    if (a.g.nz == 58) {
      if (full) hipLaunchKernelGGL((k_hevi_stage_split<T, true, 58>), dim3(nb2), dim3(64, rows), 0, s, a);
      else hipLaunchKernelGGL((k_hevi_stage_split<T, false, 58>), dim3(nb2), dim3(64, rows), 0, s, a);
    } else {
      if (full) hipLaunchKernelGGL((k_hevi_stage_split<T, true, 16>), dim3(nb2), dim3(64, rows), 0, s, a);
      else hipLaunchKernelGGL((k_hevi_stage_split<T, false, 16>), dim3(nb2), dim3(64, rows), 0, s, a);
    }
    return hipGetLastError();
  }
  if (kernel != 1 && fixed) {
    if (a.g.nz == 58) {
      if (full) hipLaunchKernelGGL((k_hevi_stage_reg<T, true, 58>), dim3(nb), dim3(64, 4), 0, s, a);
      else hipLaunchKernelGGL((k_hevi_stage_reg<T, false, 58>), dim3(nb), dim3(64, 4), 0, s, a);
    } else {
      if (full) hipLaunchKernelGGL((k_hevi_stage_reg<T, true, 16>), dim3(nb), dim3(64, 4), 0, s, a);
      else hipLaunchKernelGGL((k_hevi_stage_reg<T, false, 16>), dim3(nb), dim3(64, 4), 0, s, a);
    }
    return hipGetLastError();
  }
  if (full)
    hipLaunchKernelGGL((k_hevi_stage<T, true>), dim3(nb), dim3(64, 4), 0, s, a);
  else
    hipLaunchKernelGGL((k_hevi_stage<T, false>), dim3(nb), dim3(64, 4), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_hevi_stage<float>(const HeviArgs<float> &, bool, int, hipStream_t);
template hipError_t launch_hevi_stage<double>(const HeviArgs<double> &, bool, int, hipStream_t);

}  // namespace wx
