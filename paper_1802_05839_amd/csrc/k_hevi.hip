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

}  // namespace

template <typename T>
hipError_t launch_hevi_stage(const HeviArgs<T> &a, bool full, hipStream_t s) {
  const int nb = ((a.g.nx + 63) / 64) * ((a.g.ny + 3) / 4);
  if (full)
    hipLaunchKernelGGL((k_hevi_stage<T, true>), dim3(nb), dim3(64, 4), 0, s, a);
  else
    hipLaunchKernelGGL((k_hevi_stage<T, false>), dim3(nb), dim3(64, 4), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_hevi_stage<float>(const HeviArgs<float> &, bool, hipStream_t);
template hipError_t launch_hevi_stage<double>(const HeviArgs<double> &, bool, hipStream_t);

}  // namespace wx
