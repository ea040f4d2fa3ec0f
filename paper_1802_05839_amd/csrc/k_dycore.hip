// Dynamical core kernels: periodic halo fill and one RK3 stage.
//
// Method (readings of section "The ASUCA Weather Prediction Model", which
// fixes a C-grid finite-volume discretisation with I/J horizontal and K
// separate, and a third-order Runge-Kutta long step):
//   face values   third-order upwind, weights (-1, 5, 2)/6 toward the wind,
//                 in k centred next to the ground and lid, no flux through them;
//   mass flux     F = wind * rho*_face;
//   density       rho_new = rho_n - h div(F);
//   tracers       phi_new = phi_n + h (A + B) / rho_new with the increment form
//                 A = -sum_faces +-F (phi*_face - phi_n) / spacing and the
//                 density-weighted biharmonic B = -div(K4 rho*_face grad Lap(phi*)).
//
// GPU design (section "Architecture-Dependent Storage Order": i stride-1 on
// GPUs; K marched sequentially inside each thread as in the paper's generated
// kernels, appendix "Reduced Weather: Diffusion"):
//   * a 512-thread block owns a 64 x 8 column tile and marches k = 0..nz-1
//     (8 rows keep the re-read 2-row halo of the staged fields at 1.5x);
//   * each k-plane of rho*, theta*, q* is staged once into LDS as a 68 x 12
//     tile (2-cell halo), giving all horizontal neighbours; a 4-deep LDS ring
//     (planes k..k+3) lets the vertical stencil read k+1, k+2 and the global
//     loads of plane k+3 overlap the arithmetic of plane k, with one barrier
//     per plane;
//   * the vertical window (k-2, k-1) and the lower face flux are carried in
//     registers, so every face in k is computed once;
//   * a block's linear id is remapped so that each of the 8 XCDs works on a
//     contiguous band of tiles (neighbouring tiles share their halo rows in
//     the same L2);
//   * the output's periodic halo images are written by the cell that owns
//     them, so no separate halo pass runs between stages.
#include "wx_internal.h"

namespace wx {
namespace {

constexpr int NBUF = 4;

// Third-order upwind face value from the far-upstream, upstream and
// downstream cells: b + (2 (c - b) + (b - a)) / 6.
template <typename T>
__device__ __forceinline__ T face3(T a, T b, T c) {
  return b + (T(2) * (c - b) + (b - a)) * T(1.0 / 6.0);
}

// Both faces of a cell along one axis from the five cells m2, m1, c, p1, p2
// and the wind sign at each face, sharing the four differences:
//   upper face (c | p1): c + (2 d1 + d0)/6 if the wind is >= 0, else
//                        p1 - (2 d1 + d2)/6;
//   lower face (m1 | c): m1 + (2 d0 + dm)/6, else c - (2 d0 + d1)/6.
// Branch-free; each value is bitwise that of face3 on the same three cells,
// so the two cells sharing a face compute the same value.
template <typename T>
__device__ __forceinline__ void faces3(T m2, T m1, T c, T p1, T p2, bool up_hi, bool up_lo, T &f_hi, T &f_lo) {
  const T dm = m1 - m2, d0 = c - m1, d1 = p1 - c, d2 = p2 - p1;
  const T s6 = T(1.0 / 6.0);
  f_hi = fma(fma(T(2), d1, up_hi ? d0 : d2), up_hi ? s6 : -s6, up_hi ? c : p1);
  f_lo = fma(fma(T(2), d0, up_lo ? dm : d1), up_lo ? s6 : -s6, up_lo ? m1 : c);
}

template <typename T>
__global__ void k_halo(T *f0, T *f1, T *f2, T *f3, T *f4, int nx, int ny, unsigned sj,
                       unsigned sk, unsigned origin) {
  const int ring = 4 * (nx + 4) + 4 * ny;
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ring) return;
  T *f = blockIdx.z == 0 ? f0 : blockIdx.z == 1 ? f1 : blockIdx.z == 2 ? f2 : blockIdx.z == 3 ? f3 : f4;
  int i, j;
  if (r < 4 * (nx + 4)) {
    const int row = r / (nx + 4);
    j = row < 2 ? row - 2 : ny + row - 2;
    i = r % (nx + 4) - 2;
  } else {
    const int rr = r - 4 * (nx + 4);
    j = rr >> 2;
    const int c = rr & 3;
    i = c < 2 ? c - 2 : nx + c - 2;
  }
  const int si = (i + nx) % nx, sjj = (j + ny) % ny;
  const unsigned pl = blockIdx.y * sk + origin;
  stg(f, pl + unsigned(i + j * int(sj)), ldg(f, pl + unsigned(si + sjj * int(sj))));
}

// BX x BY tile (production 64 x 8; the other shapes are the block-shape
// ablation, selected at run time through WX_PARAM_STAGE_TILE).
template <typename T, int STAGE, int BX, int BY>
__global__ __launch_bounds__(BX * BY) void k_stage(StageArgs<T> a) {
  constexpr int TW = BX + 4, TH = BY + 4, TN = TW * TH;  // tile with its 2-cell halo
  constexpr int NT = BX * BY;
  constexpr int NLOAD = (TN + NT - 1) / NT;               // tile elements per thread
  __shared__ T s_r[NBUF][TN];
  __shared__ T s_t[NBUF][TN];
  __shared__ T s_q[NBUF][TN];

  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
  const int L = a.reverse ? xcd_remap_rev(blockIdx.x, a.nblocks) : xcd_remap(blockIdx.x, a.nblocks);
  const int i0 = (L % a.nbx) * BX, j0 = (L / a.nbx) * BY;
  const int i = i0 + tx, j = j0 + ty;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const unsigned sj = a.g.sj, sk = a.g.sk;
  const bool active = (i < nx) && (j < ny);

  // This thread's share of the (BX+4) x (BY+4) plane tile.
  unsigned toff[NLOAD];
  bool tok[NLOAD];
#pragma unroll
  for (int n = 0; n < NLOAD; ++n) {
    const int e = tid + n * NT;
    const int gi = i0 - 2 + e % TW, gj = j0 - 2 + e / TW;
    tok[n] = (e < TN) && (gi < nx + 2) && (gj < ny + 2);
    toff[n] = unsigned(int(a.g.origin) + gi + gj * int(sj));
  }
  T pr[NLOAD], pt[NLOAD], pq[NLOAD];
  auto fetch = [&](int p) {
    const unsigned base = unsigned(p) * sk;
#pragma unroll
    for (int n = 0; n < NLOAD; ++n) {
      pr[n] = tok[n] ? ldg(a.in_r, base + toff[n]) : T(0);
      pt[n] = tok[n] ? ldg(a.in_t, base + toff[n]) : T(0);
      pq[n] = tok[n] ? ldg(a.in_q, base + toff[n]) : T(0);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int n = 0; n < NLOAD; ++n) {
      const int e = tid + n * NT;
      if (e < TN) {
        s_r[buf][e] = pr[n];
        s_t[buf][e] = pt[n];
        s_q[buf][e] = pq[n];
      }
    }
  };

  const int npre = nz < 3 ? nz : 3;
  for (int p = 0; p < npre; ++p) {
    fetch(p);
    stash(p);
  }
  if (nz > 3) fetch(3);
  __syncthreads();

  const int c0 = (ty + 2) * TW + (tx + 2);
  // vertical window of this column: planes k-2 .. k+2
  T rm2 = 0, rm1 = 0, r0 = s_r[0][c0], rp1 = s_r[1][c0], rp2 = 0;
  T tm2 = 0, tm1 = 0, t0 = s_t[0][c0], tp1 = s_t[1][c0], tp2 = 0;
  T qm2 = 0, qm1 = 0, q0 = s_q[0][c0], qp1 = s_q[1][c0], qp2 = 0;
  (void)rm2; (void)tm2; (void)qm2;
  // flux and face values at the face below the current level
  T fzb = 0, tfb = 0, qfb = 0;

  const unsigned col = a.g.origin + unsigned(i) + unsigned(j) * sj;
  // west, south and upper-face winds through shifted (uniform) base
  // pointers, so that every load of a level uses the same vector offset gc
  const T *uw = plane(a.u, -1), *vs = plane(a.v, -(long long)sj), *wu = plane(a.w, (long long)sk);
  T wb = 0;
  const T h = a.h, rdx = a.rdx, k4 = a.k4;
  const T r2 = rdx * rdx;

  for (int k = 0; k < nz; ++k) {
    if (k > 0) __syncthreads();
    const int b = k & (NBUF - 1);
    if (k + 2 < nz) {
      const int b2 = (k + 2) & (NBUF - 1);
      rp2 = s_r[b2][c0];
      tp2 = s_t[b2][c0];
      qp2 = s_q[b2][c0];
    }
    if (active) {
      const T *R = s_r[b] + c0;
      const T *Th = s_t[b] + c0;
      const T *Q = s_q[b] + c0;
      const unsigned gc = col + unsigned(k) * sk;
      const T uE = ldg(a.u, gc), uW = ldg(uw, gc), vN = ldg(a.v, gc), vS = ldg(vs, gc);
      const T wt = (k + 1 < nz) ? ldg(wu, gc) : T(0);
      const T rdz = a.rdz[k];

      // --- density: face values and mass fluxes
      const T rxm2 = R[-2], rxm1 = R[-1], rxp1 = R[1], rxp2 = R[2];
      const T rym2 = R[-2 * TW], rym1 = R[-TW], ryp1 = R[TW], ryp2 = R[2 * TW];
      const bool upE = uE >= T(0), upW = uW >= T(0), upN = vN >= T(0), upS = vS >= T(0);
      T rfE, rfW, rfN, rfS;
      faces3(rxm2, rxm1, r0, rxp1, rxp2, upE, upW, rfE, rfW);
      faces3(rym2, rym1, r0, ryp1, ryp2, upN, upS, rfN, rfS);
      T rfT = 0, tfT = 0, qfT = 0;
      const bool top = (k + 1 >= nz);
      const bool centred = (k == 0) || (k + 2 == nz);
      if (!top) {
        if (centred) {
          rfT = r0 + (rp1 - r0) * T(0.5);
          tfT = t0 + (tp1 - t0) * T(0.5);
          qfT = q0 + (qp1 - q0) * T(0.5);
        } else if (wt >= T(0)) {
          rfT = face3(rm1, r0, rp1);
          tfT = face3(tm1, t0, tp1);
          qfT = face3(qm1, q0, qp1);
        } else {
          rfT = face3(rp2, rp1, r0);
          tfT = face3(tp2, tp1, t0);
          qfT = face3(qp2, qp1, q0);
        }
      }
      // mass fluxes, pre-scaled by 1/dx or 1/dz (shared by the three fields;
      // the neighbour that shares a face computes the same value bitwise)
      const T FE = uE * rfE * rdx, FW = uW * rfW * rdx, FN = vN * rfN * rdx, FS = vS * rfS * rdx;
      const T fzT = top ? T(0) : wt * rfT;
      const T FT = fzT * rdz, FB = fzb * rdz;
      const T div = ((FE - FW) + (FN - FS)) + (FT - FB);

      T br, bt, bq;
      if (STAGE == 1) {
        br = r0;
        bt = t0;
        bq = q0;
      } else {
        br = ldg(a.bs_r, gc);
        bt = ldg(a.bs_t, gc);
        bq = ldg(a.bs_q, gc);
      }
      const T rnew = br - h * div;
      const T hr = h * fast_rcp(rnew);

      // twice the density at the four horizontal faces, and their sum
      const T rhE = r0 + rxp1, rhW = rxm1 + r0, rhN = r0 + ryp1, rhS = rym1 + r0;
      const T rhSum = (rhE + rhW) + (rhN + rhS);

      // phi_new = base + h (A + B) / rho_new with
      //   A = -sum_faces +-F (phi_face - base) / spacing            (increment form)
      //   B = -div(K4 rho_face grad Lap phi)
      //     = -(K4 / (2 dx^4)) [sum_nb 2 rho_face L_nb - (sum 2 rho_face) L_c]
      // where L = (sum of the four neighbours) - 4 phi is dx^2 times the
      // Laplacian; constant phi gives A = B = 0 exactly.
      const T cB = k4 * T(0.5) * r2 * r2;
      auto tracer = [&](const T *P, T pc, T fzfT, T fzfB, T base) -> T {
        const T xm2 = P[-2], xm1 = P[-1], xp1 = P[1], xp2 = P[2];
        const T ym2 = P[-2 * TW], ym1 = P[-TW], yp1 = P[TW], yp2 = P[2 * TW];
        const T dpp = P[TW + 1], dpm = P[-TW + 1], dmp = P[TW - 1], dmm = P[-TW - 1];
        T fE, fW, fN, fS;
        faces3(xm2, xm1, pc, xp1, xp2, upE, upW, fE, fW);
        faces3(ym2, ym1, pc, yp1, yp2, upN, upS, fN, fS);
        T adv = FE * (fE - base);
        adv -= FW * (fW - base);
        adv += FN * (fN - base);
        adv -= FS * (fS - base);
        adv += FT * (fzfT - base);
        adv -= FB * (fzfB - base);
        const T lc = ((xp1 + xm1) + (yp1 + ym1)) - T(4) * pc;
        const T le = ((xp2 + pc) + (dpp + dpm)) - T(4) * xp1;
        const T lw = ((pc + xm2) + (dmp + dmm)) - T(4) * xm1;
        const T ln = ((dpp + dmp) + (yp2 + pc)) - T(4) * yp1;
        const T ls = ((dpm + dmm) + (pc + ym2)) - T(4) * ym1;
        T bs = rhE * le;
        bs += rhW * lw;
        bs += rhN * ln;
        bs += rhS * ls;
        bs -= rhSum * lc;
        return base - hr * (adv + cB * bs);
      };
      const T tnew = tracer(Th, t0, tfT, tfb, bt);
      const T qnew = tracer(Q, q0, qfT, qfb, bq);

      // store the cell and its periodic images in the halo ring.  Stage 3's
      // output (the new state) is read next by the physics launch from its
      // first column on, which the memory-side cache no longer holds once
      // the whole grid has been written, so it is stored non-temporally
      // (1.38 -> 1.36 ms); on stages 1 and 2 the hint costs 7%
      if (STAGE == 3) {
        __builtin_nontemporal_store(rnew, a.out_r + gc);
        __builtin_nontemporal_store(tnew, a.out_t + gc);
        __builtin_nontemporal_store(qnew, a.out_q + gc);
      } else {
        stg(a.out_r, gc, rnew);
        stg(a.out_t, gc, tnew);
        stg(a.out_q, gc, qnew);
      }
      const int di = i < 2 ? nx : (i >= nx - 2 ? -nx : 0);
      const int dj = j < 2 ? ny * int(sj) : (j >= ny - 2 ? -ny * int(sj) : 0);
      if (di != 0) {
        stg(a.out_r, gc + di, rnew);
        stg(a.out_t, gc + di, tnew);
        stg(a.out_q, gc + di, qnew);
      }
      if (dj != 0) {
        stg(a.out_r, gc + dj, rnew);
        stg(a.out_t, gc + dj, tnew);
        stg(a.out_q, gc + dj, qnew);
        if (di != 0) {
          stg(a.out_r, gc + dj + di, rnew);
          stg(a.out_t, gc + dj + di, tnew);
          stg(a.out_q, gc + dj + di, qnew);
        }
      }
      fzb = fzT;
      tfb = tfT;
      qfb = qfT;
      wb = wt;
    }
    // shift the vertical window
    rm2 = rm1; rm1 = r0; r0 = rp1; rp1 = rp2;
    tm2 = tm1; tm1 = t0; t0 = tp1; tp1 = tp2;
    qm2 = qm1; qm1 = q0; q0 = qp1; qp1 = qp2;
    // move plane k+3 into the ring and start loading plane k+4
    if (k + 3 < nz) {
      stash((k + 3) & (NBUF - 1));
      if (k + 4 < nz) fetch(k + 4);
    }
  }
  (void)wb;
}

// The same stage with every face value, mass flux and Laplacian computed
// once per tile instead of once per adjacent cell.  Per level:
//   phase A (all 512 threads, after the plane is in LDS): the 65 x 8 x-faces
//     and 64 x 9 y-faces of the tile (upwind rho, theta, q face values, the
//     mass flux (wind * rho_face) / dx and the density pair sum rho_l + rho_r
//     of the biharmonic flux) and the Laplacians of theta and q on the 66 x 10
//     cells of the tile and its one-cell rim, into LDS;
//   phase B (one thread per cell): the vertical face in registers as before,
//     then the flux divergence and the updates from the LDS face arrays.
// Each face is formed from the same operands in the same order as the per-
// cell kernel forms it (that kernel's two neighbours already computed it
// bitwise alike), so the two kernels give the same bits.  The plane ring is
// three deep: a plane is only read horizontally in phase A of its own level,
// and each thread copies its own column of a plane into registers (the
// vertical window) right after the plane arrives.
constexpr int SF_BX = 64, SF_BY = 8, SF_TW = SF_BX + 4, SF_TH = SF_BY + 4, SF_TN = SF_TW * SF_TH;
constexpr int SF_NT = SF_BX * SF_BY, SF_NLOAD = (SF_TN + SF_NT - 1) / SF_NT, SF_NBUF = 3;
constexpr int SF_XF = SF_BX + 1;           // x-faces per row
constexpr int SF_LW = SF_BX + 2, SF_LH = SF_BY + 2, SF_LN = SF_LW * SF_LH;   // Laplacian region

template <typename T, int STAGE>
__global__ __launch_bounds__(SF_NT, 6) void k_stage_sf(StageArgs<T> a) {
  __shared__ T s_r[SF_NBUF][SF_TN];
  __shared__ T s_t[SF_NBUF][SF_TN];
  __shared__ T s_q[SF_NBUF][SF_TN];
  // x-face arrays [row][face], y-face arrays [face row][column], Laplacians [row][col]
  __shared__ T xF[SF_BY][SF_XF], xR[SF_BY][SF_XF], xT[SF_BY][SF_XF], xQ[SF_BY][SF_XF];
  __shared__ T yF[SF_BY + 1][SF_BX], yR[SF_BY + 1][SF_BX], yT[SF_BY + 1][SF_BX], yQ[SF_BY + 1][SF_BX];
  __shared__ T lT[SF_LN], lQ[SF_LN];

  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * SF_BX + tx;
  const int L = xcd_remap(blockIdx.x, a.nblocks);
  const int i0 = (L % a.nbx) * SF_BX, j0 = (L / a.nbx) * SF_BY;
  const int i = i0 + tx, j = j0 + ty;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const unsigned sj = a.g.sj, sk = a.g.sk;
  const bool active = (i < nx) && (j < ny);

  unsigned toff[SF_NLOAD];
  bool tok[SF_NLOAD];
#pragma unroll
  for (int n = 0; n < SF_NLOAD; ++n) {
    const int e = tid + n * SF_NT;
    const int gi = i0 - 2 + e % SF_TW, gj = j0 - 2 + e / SF_TW;
    tok[n] = (e < SF_TN) && (gi < nx + 2) && (gj < ny + 2);
    toff[n] = unsigned(int(a.g.origin) + gi + gj * int(sj));
  }
  T pr[SF_NLOAD], pt[SF_NLOAD], pq[SF_NLOAD];
  auto fetch = [&](int p) {
    const unsigned base = unsigned(p) * sk;
#pragma unroll
    for (int n = 0; n < SF_NLOAD; ++n) {
      pr[n] = tok[n] ? ldg(a.in_r, base + toff[n]) : T(0);
      pt[n] = tok[n] ? ldg(a.in_t, base + toff[n]) : T(0);
      pq[n] = tok[n] ? ldg(a.in_q, base + toff[n]) : T(0);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int n = 0; n < SF_NLOAD; ++n) {
      const int e = tid + n * SF_NT;
      if (e < SF_TN) {
        s_r[buf][e] = pr[n];
        s_t[buf][e] = pt[n];
        s_q[buf][e] = pq[n];
      }
    }
  };

  const T rdx = a.rdx, h = a.h, k4 = a.k4;
  const T r2 = rdx * rdx;
  const T cB = k4 * T(0.5) * r2 * r2;
  const unsigned origin = a.g.origin;

  // x-face x of row y: between tile columns x+1 (left) and x+2 (right); the
  // wind uu is u at the east face of the left cell, i = i0 + x - 1
  auto xface = [&](const T *R, const T *Th, const T *Q, int x, int y, T uu) {
    const bool up = uu >= T(0);
    const int c = (y + 2) * SF_TW + (x + 1);      // left cell
    const T s6 = T(1.0 / 6.0);
    auto f = [&](const T *P) {
      const T pa = P[c - 1], pb = P[c], pc = P[c + 1], pd = P[c + 2];
      const T d0 = pb - pa, d1 = pc - pb, d2 = pd - pc;
      return fma(fma(T(2), d1, up ? d0 : d2), up ? s6 : -s6, up ? pb : pc);
    };
    const T rf = f(R);
    xF[y][x] = uu * rf * rdx;
    xR[y][x] = R[c] + R[c + 1];
    xT[y][x] = f(Th);
    xQ[y][x] = f(Q);
  };
  // y-face y of column x: between tile rows y+1 (lower) and y+2 (upper); the
  // wind vv is v at the north face of the lower cell, j = j0 + y - 1
  auto yface = [&](const T *R, const T *Th, const T *Q, int x, int y, T vv) {
    const bool up = vv >= T(0);
    const int c = (y + 1) * SF_TW + (x + 2);      // lower cell
    const T s6 = T(1.0 / 6.0);
    auto f = [&](const T *P) {
      const T pa = P[c - SF_TW], pb = P[c], pc = P[c + SF_TW], pd = P[c + 2 * SF_TW];
      const T d0 = pb - pa, d1 = pc - pb, d2 = pd - pc;
      return fma(fma(T(2), d1, up ? d0 : d2), up ? s6 : -s6, up ? pb : pc);
    };
    const T rf = f(R);
    yF[y][x] = vv * rf * rdx;
    yR[y][x] = R[c] + R[c + SF_TW];
    yT[y][x] = f(Th);
    yQ[y][x] = f(Q);
  };
  // Laplacian (times dx^2) of theta and q at region cell n (tile cell
  // (n % 66 + 1, n / 66 + 1)): ((E + W) + (N + S)) - 4 C
  auto lap = [&](const T *Th, const T *Q, int n) {
    const int c = (n / SF_LW + 1) * SF_TW + (n % SF_LW + 1);
    lT[n] = ((Th[c + 1] + Th[c - 1]) + (Th[c + SF_TW] + Th[c - SF_TW])) - T(4) * Th[c];
    lQ[n] = ((Q[c + 1] + Q[c - 1]) + (Q[c + SF_TW] + Q[c - SF_TW])) - T(4) * Q[c];
  };

  // the winds of this thread's faces (its own x- and y-face, and the extra
  // 65th x-face of a row or 9th y-face row for the first 72 threads), loaded
  // one level ahead
  auto woff = [&](int gi, int gj, bool &ok) {
    ok = gi <= nx + 1 && gj <= ny + 1;
    return origin + unsigned(gi + gj * int(sj));
  };
  bool xok, yok, eok = false;
  const unsigned xo = woff(i0 + tx - 1, j0 + ty, xok), yo = woff(i0 + tx, j0 + ty - 1, yok);
  const bool ex = tid < SF_BY, ey = !ex && tid < SF_BY + SF_BX;
  const unsigned eo = ex ? woff(i0 + SF_BX - 1, j0 + tid, eok) : ey ? woff(i0 + tid - SF_BY, j0 + SF_BY - 1, eok) : 0u;
  const T *ew = ex ? a.u : a.v;
  T ux = 0, vy = 0, we = 0;
  auto fetch_winds = [&](unsigned kk) {
    ux = xok ? ldg(a.u, kk + xo) : T(0);
    vy = yok ? ldg(a.v, kk + yo) : T(0);
    we = eok ? ldg(ew, kk + eo) : T(0);
  };
  fetch_winds(0u);

  // prologue: planes 0, 1, 2 into the ring, plane 3 in flight
  const int npre = nz < 3 ? nz : 3;
  for (int p = 0; p < npre; ++p) {
    fetch(p);
    stash(p);
  }
  if (nz > 3) fetch(3);
  __syncthreads();

  const int c0 = (ty + 2) * SF_TW + (tx + 2);
  T rm1 = 0, r0 = s_r[0][c0], rp1 = nz > 1 ? s_r[1][c0] : T(0), rp2 = 0;
  T tm1 = 0, t0 = s_t[0][c0], tp1 = nz > 1 ? s_t[1][c0] : T(0), tp2 = 0;
  T qm1 = 0, q0 = s_q[0][c0], qp1 = nz > 1 ? s_q[1][c0] : T(0), qp2 = 0;
  T fzb = 0, tfb = 0, qfb = 0;
  const unsigned col = origin + unsigned(i) + unsigned(j) * sj;
  const T *wu = plane(a.w, (long long)sk);

  for (int k = 0; k < nz; ++k) {
    const int b = k % SF_NBUF;
    const T *R = s_r[b], *Th = s_t[b], *Q = s_q[b];
    if (k + 2 < nz) {
      const int b2 = (k + 2) % SF_NBUF;
      rp2 = s_r[b2][c0];
      tp2 = s_t[b2][c0];
      qp2 = s_q[b2][c0];
    }
    // ---- phase A
    const unsigned kk = unsigned(k) * sk;
    const T uxk = ux, vyk = vy, wek = we;
    if (k + 1 < nz) fetch_winds(kk + sk);
    xface(R, Th, Q, tx, ty, uxk);
    yface(R, Th, Q, tx, ty, vyk);
    lap(Th, Q, tid);
    if (ex) {
      xface(R, Th, Q, SF_BX, tid, wek);
    } else if (ey) {
      yface(R, Th, Q, tid - SF_BY, SF_BY, wek);
    } else if (tid < SF_BY + SF_BX + (SF_LN - SF_NT)) {
      lap(Th, Q, SF_NT + tid - SF_BY - SF_BX);
    }
    __syncthreads();
    // the plane of level k is no longer read: plane k+3 takes its buffer and
    // plane k+4 starts loading
    if (k + 3 < nz) {
      stash((k + 3) % SF_NBUF);
      if (k + 4 < nz) fetch(k + 4);
    }
    // ---- phase B
    if (active) {
      const unsigned gc = col + kk;
      const T wt = (k + 1 < nz) ? ldg(wu, gc) : T(0);
      const T rdz = a.rdz[k];
      T rfT = 0, tfT = 0, qfT = 0;
      const bool top = (k + 1 >= nz);
      const bool centred = (k == 0) || (k + 2 == nz);
      if (!top) {
        if (centred) {
          rfT = r0 + (rp1 - r0) * T(0.5);
          tfT = t0 + (tp1 - t0) * T(0.5);
          qfT = q0 + (qp1 - q0) * T(0.5);
        } else if (wt >= T(0)) {
          rfT = face3(rm1, r0, rp1);
          tfT = face3(tm1, t0, tp1);
          qfT = face3(qm1, q0, qp1);
        } else {
          rfT = face3(rp2, rp1, r0);
          tfT = face3(tp2, tp1, t0);
          qfT = face3(qp2, qp1, q0);
        }
      }
      const T FE = xF[ty][tx + 1], FW = xF[ty][tx], FN = yF[ty + 1][tx], FS = yF[ty][tx];
      const T fzT = top ? T(0) : wt * rfT;
      const T FT = fzT * rdz, FB = fzb * rdz;
      const T div = ((FE - FW) + (FN - FS)) + (FT - FB);
      T br, bt, bq;
      if (STAGE == 1) {
        br = r0;
        bt = t0;
        bq = q0;
      } else {
        br = ldg(a.bs_r, gc);
        bt = ldg(a.bs_t, gc);
        bq = ldg(a.bs_q, gc);
      }
      const T rnew = br - h * div;
      const T hr = h * fast_rcp(rnew);
      const T rhE = xR[ty][tx + 1], rhW = xR[ty][tx], rhN = yR[ty + 1][tx], rhS = yR[ty][tx];
      const T rhSum = (rhE + rhW) + (rhN + rhS);
      const int lc0 = (ty + 1) * SF_LW + (tx + 1);
      auto tracer = [&](const T (*XP)[SF_XF], const T (*YP)[SF_BX], const T *LP, T fzfT, T fzfB, T base) -> T {
        const T fE = XP[ty][tx + 1], fW = XP[ty][tx], fN = YP[ty + 1][tx], fS = YP[ty][tx];
        T adv = FE * (fE - base);
        adv -= FW * (fW - base);
        adv += FN * (fN - base);
        adv -= FS * (fS - base);
        adv += FT * (fzfT - base);
        adv -= FB * (fzfB - base);
        const T lc = LP[lc0], le = LP[lc0 + 1], lw = LP[lc0 - 1], ln = LP[lc0 + SF_LW], ls = LP[lc0 - SF_LW];
        T bs = rhE * le;
        bs += rhW * lw;
        bs += rhN * ln;
        bs += rhS * ls;
        bs -= rhSum * lc;
        return base - hr * (adv + cB * bs);
      };
      const T tnew = tracer(xT, yT, lT, tfT, tfb, bt);
      const T qnew = tracer(xQ, yQ, lQ, qfT, qfb, bq);
      stg(a.out_r, gc, rnew);
      stg(a.out_t, gc, tnew);
      stg(a.out_q, gc, qnew);
      const int di = i < 2 ? nx : (i >= nx - 2 ? -nx : 0);
      const int dj = j < 2 ? ny * int(sj) : (j >= ny - 2 ? -ny * int(sj) : 0);
      if (di != 0) {
        stg(a.out_r, gc + di, rnew);
        stg(a.out_t, gc + di, tnew);
        stg(a.out_q, gc + di, qnew);
      }
      if (dj != 0) {
        stg(a.out_r, gc + dj, rnew);
        stg(a.out_t, gc + dj, tnew);
        stg(a.out_q, gc + dj, qnew);
        if (di != 0) {
          stg(a.out_r, gc + dj + di, rnew);
          stg(a.out_t, gc + dj + di, tnew);
          stg(a.out_q, gc + dj + di, qnew);
        }
      }
      fzb = fzT;
      tfb = tfT;
      qfb = qfT;
    }
    rm1 = r0; r0 = rp1; rp1 = rp2;
    tm1 = t0; t0 = tp1; tp1 = tp2;
    qm1 = q0; q0 = qp1; qp1 = qp2;
    // phase B is done with the face arrays and plane k+3 is in the ring
    __syncthreads();
  }
}

}  // namespace

template <typename T>
hipError_t launch_halo(T *const *fields, int nf, int nplanes, const Geom &g, hipStream_t s) {
  if (nf < 1 || nf > 5) return hipErrorInvalidValue;
  const int ring = 4 * (g.nx + 4) + 4 * g.ny;
  dim3 grid((ring + 255) / 256, nplanes, nf);
  T *f[5];
  for (int n = 0; n < 5; ++n) f[n] = fields[n < nf ? n : 0];
  hipLaunchKernelGGL(k_halo<T>, grid, dim3(256), 0, s, f[0], f[1], f[2], f[3], f[4], g.nx, g.ny,
                     g.sj, g.sk, g.origin);
  return hipGetLastError();
}

template <typename T, int BX, int BY>
void launch_stage_shape(const StageArgs<T> &a, int stage, hipStream_t s) {
  const dim3 block(BX, BY), grid(a.nblocks);
  if (stage == 1)
    hipLaunchKernelGGL((k_stage<T, 1, BX, BY>), grid, block, 0, s, a);
  else if (stage == 2)
    hipLaunchKernelGGL((k_stage<T, 2, BX, BY>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((k_stage<T, 3, BX, BY>), grid, block, 0, s, a);
}

template <typename T>
hipError_t launch_stage(const StageArgs<T> &a, int stage, int tile, hipStream_t s) {
  if (tile == STAGE_TILE_SHARED) {
    if (a.nbx != (a.g.nx + SF_BX - 1) / SF_BX || a.nblocks != a.nbx * ((a.g.ny + SF_BY - 1) / SF_BY))
      return hipErrorInvalidValue;
    const dim3 block(SF_BX, SF_BY), grid(a.nblocks);
    if (stage == 1)
      hipLaunchKernelGGL((k_stage_sf<T, 1>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((k_stage_sf<T, 2>), grid, block, 0, s, a);
    return hipGetLastError();
  }
  const StageShape sh = stage_shape(tile);
  if (sh.bx == 0) return hipErrorInvalidValue;
  if (a.nbx != (a.g.nx + sh.bx - 1) / sh.bx || a.nblocks != a.nbx * ((a.g.ny + sh.by - 1) / sh.by))
    return hipErrorInvalidValue;
  switch (tile) {
    case 0: launch_stage_shape<T, 64, 8>(a, stage, s); break;
    case 1: launch_stage_shape<T, 64, 4>(a, stage, s); break;
    case 2: launch_stage_shape<T, 64, 12>(a, stage, s); break;
    case 3: launch_stage_shape<T, 32, 16>(a, stage, s); break;
    case 4: launch_stage_shape<T, 128, 4>(a, stage, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_halo<float>(float *const *, int, int, const Geom &, hipStream_t);
template hipError_t launch_halo<double>(double *const *, int, int, const Geom &, hipStream_t);
template hipError_t launch_stage<float>(const StageArgs<float> &, int, int, hipStream_t);
template hipError_t launch_stage<double>(const StageArgs<double> &, int, int, hipStream_t);

}  // namespace wx
