// The paper's reduced weather application (section "Reduced Weather
// Application" and the appendix sources of its diffusion, physical processes,
// radiation, heat exchange and time integration), one fused kernel per time
// step.
//
// Method (FP64 as printed): a step applies the column physics to every column
// (radiation adds 0.1 to every level, then the bottom level loses 0.01 times
// its excess over the surface value and the top level 0.01 times its excess
// over the boundary-layer value) and then one explicit-Euler diffusion step
// into the other array:
//   interior column, inner level:  E (1 - 6 nu) + nu (i-1 + i+1 + j-1 + j+1 + k-1 + k+1)
//   interior column, level 1 / nz: E (1 - 5 nu) + nu (i-1 + i+1 + j-1 + j+1 + the one vertical)
//   ring row j = 0 / ny+1:         E (1 - 2 nu) + nu (inner row + opposite ring row)
//   ring column i = 0 / nx+1:      E (1 - 2 nu) + nu (inner column + opposite ring column),
//                                  corners included (the column rule is written last).
// Every sum is taken in that order and no multiply-add is fused, so the result
// is the printed program's to the last bit.
//
// GPU design: the physics is applied on the fly to every value the diffusion
// reads (it is pointwise in each column apart from its own surface and
// boundary-layer values), so a step reads the field once and writes it once:
// 16 B per cell.  A 64 x 8 block of threads owns a tile of interior columns
// (i fastest, coalesced rows) and marches a chunk of levels.  Each level's
// 66 x 10 tile (the 64 x 8 cells and their one-cell rim) is loaded once with
// coalesced reads, passed through the physics and kept in a 4-deep LDS ring,
// so a cell's six neighbours and its vertical window are LDS reads, and the
// loads of level k+2 are in flight while level k is computed (one barrier per
// level).  Tiles of one level chunk are numbered i-fastest and mapped XCD by
// XCD, so the rows shared by j-neighbouring tiles meet in one L2.  The ring
// cells (about 1% of a large grid) take extra blocks of the same launch, one
// cell per thread, so no wavefront mixes the two rules.
#include "wx_internal.h"

#pragma clang fp contract(off)

namespace wx {
namespace {

constexpr int KIJ_BX = 64, KIJ_BY = 4;   // the KIJ kernel's thread block (one thread per column)

struct RwArgs {
  const double *e;
  double *out;
  const double *surf, *pbl;      // [ny+2][nx+2]
  int nx, ny, nz, kchunk, nchunk;
  int tiles_x, tiles_y;          // interior tiles (i = 1..nx, j = 1..ny)
  double nu, c6, c5, c2;
};

// The column physics of level k applied to the value v of column ij.
__device__ __forceinline__ double phys(const RwArgs &a, double v, int k, unsigned ij) {
  double r = v + 0.1;
  if (k == 0) {
    const double lost = 0.01 * (r - a.surf[ij]);
    r = r - lost;
  }
  if (k == a.nz - 1) {
    const double lost = 0.01 * (r - a.pbl[ij]);
    r = r - lost;
  }
  return r;
}

// Ring columns: i = 0 or nx + 1 (every j, corners included), then j = 0 or
// ny + 1 for i = 1..nx.  Column c of the 2 (ny + 2) + 2 nx ring columns.
__device__ __forceinline__ void ring_column(int c, int nx, int ny, int &i, int &j) {
  const int ncol_i = ny + 2;
  if (c < 2 * ncol_i) {
    i = c < ncol_i ? 0 : nx + 1;
    j = c < ncol_i ? c : c - ncol_i;
  } else {
    c -= 2 * ncol_i;
    j = c < nx ? 0 : ny + 1;
    i = 1 + (c < nx ? c : c - nx);
  }
}

// RW_BX x RW_BY thread block: 64 x 8 in production; the paper's 32 x 16 and
// its compiler's default 128 x 1, and 64 x 4, 128 x 4 are the block-size
// ablation (same arithmetic per cell, so the same bits).
template <int RW_BX, int RW_BY>
__global__ __launch_bounds__(RW_BX *RW_BY) void k_rw_step(RwArgs a) {
  constexpr int RW_TW = RW_BX + 2, RW_TH = RW_BY + 2, RW_TN = RW_TW * RW_TH;   // level tile with its rim
  constexpr int RW_NT = RW_BX * RW_BY, RW_NLOAD = (RW_TN + RW_NT - 1) / RW_NT;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const unsigned sj = unsigned(nx + 2), sk = sj * unsigned(ny + 2);
  const double nu = a.nu;
  const int nint = a.tiles_x * a.tiles_y * a.nchunk;

  if (int(blockIdx.x) >= nint) {
    // ---- ring cells, one per thread: the one-dimensional ring rule (the
    // inner neighbour, then the opposite ring cell)
    const int nring = 2 * (ny + 2) + 2 * nx;
    const int r = (int(blockIdx.x) - nint) * (RW_BX * RW_BY) + int(threadIdx.y * RW_BX + threadIdx.x);
    if (r >= nring * nz) return;
    const int k = r / nring;
    int i, j;
    ring_column(r % nring, nx, ny, i, j);
    const unsigned ij = unsigned(i) + unsigned(j) * sj;
    unsigned inner, opp;
    if (i == 0 || i == nx + 1) {
      inner = i == 0 ? ij + 1 : ij - 1;
      opp = i == 0 ? ij + unsigned(nx + 1) : ij - unsigned(nx + 1);
    } else {
      inner = j == 0 ? ij + sj : ij - sj;
      opp = j == 0 ? ij + unsigned(ny + 1) * sj : ij - unsigned(ny + 1) * sj;
    }
    const unsigned o = unsigned(k) * sk;
    const double c = phys(a, a.e[o + ij], k, ij);
    const double ni = phys(a, a.e[o + inner], k, inner);
    const double no = phys(a, a.e[o + opp], k, opp);
    a.out[o + ij] = c * a.c2 + nu * (ni + no);
    return;
  }

  // ---- interior columns: a tile marching a chunk of levels; each level's
  // plane tile with its one-cell rim (after physics) staged in a 4-deep LDS ring
  __shared__ double sp[4][RW_TH][RW_TW];
  const int ntile = a.tiles_x * a.tiles_y;
  const int L = xcd_remap(blockIdx.x, nint);
  const int chunk = L / ntile, t = L % ntile;
  const int i0 = 1 + (t % a.tiles_x) * RW_BX, j0 = 1 + (t / a.tiles_x) * RW_BY;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * RW_BX + tx;
  const int i = i0 + tx, j = j0 + ty;
  const bool active = i <= nx && j <= ny;
  const int k0 = chunk * a.kchunk, k1 = min(nz, k0 + a.kchunk);
  const double *__restrict__ E = a.e;
  double *__restrict__ OUT = a.out;
  // this thread's share of the plane tile: elements tid, tid + RW_NT, ...
  unsigned goff[RW_NLOAD];
  bool gok[RW_NLOAD];
#pragma unroll
  for (int n = 0; n < RW_NLOAD; ++n) {
    const int e = tid + n * RW_NT;
    const int gi = i0 - 1 + e % RW_TW, gj = j0 - 1 + e / RW_TW;
    gok[n] = e < RW_TN && gi <= nx + 1 && gj <= ny + 1;
    goff[n] = gok[n] ? unsigned(gi) + unsigned(gj) * sj : 0u;
  }
  double pv[RW_NLOAD];
  auto fetch = [&](int k) {
#pragma unroll
    for (int n = 0; n < RW_NLOAD; ++n) pv[n] = gok[n] ? E[unsigned(k) * sk + goff[n]] : 0.0;
  };
  auto stash = [&](int k) {
#pragma unroll
    for (int n = 0; n < RW_NLOAD; ++n) {
      const int e = tid + n * RW_NT;
      if (e < RW_TN) sp[k & 3][e / RW_TW][e % RW_TW] = gok[n] ? phys(a, pv[n], k, goff[n]) : 0.0;
    }
  };
  for (int k = (k0 > 0 ? k0 - 1 : k0); k <= k0 + 1 && k < nz; ++k) {
    fetch(k);
    stash(k);
  }
  __syncthreads();
  const int r = ty + 1, c = tx + 1;
  for (int k = k0; k < k1; ++k) {
    const bool more = k + 2 < nz && k + 2 <= k1;
    if (more) fetch(k + 2);
    if (active) {
      const double (*P)[RW_TW] = sp[k & 3];
      const double pc = P[r][c];
      double sum = P[r][c - 1] + P[r][c + 1];
      sum = sum + P[r - 1][c];
      sum = sum + P[r + 1][c];
      double res;
      if (k == 0) {
        sum = sum + sp[(k + 1) & 3][r][c];
        res = pc * a.c5 + nu * sum;
      } else if (k == nz - 1) {
        sum = sum + sp[(k - 1) & 3][r][c];
        res = pc * a.c5 + nu * sum;
      } else {
        sum = sum + sp[(k - 1) & 3][r][c];
        sum = sum + sp[(k + 1) & 3][r][c];
        res = pc * a.c6 + nu * sum;
      }
      OUT[unsigned(k) * sk + unsigned(i) + unsigned(j) * sj] = res;
    }
    if (more) stash(k + 2);
    __syncthreads();
  }
}

// The same step on the KIJ storage order (k fastest, then i, then j: element
// (i, j, k) at (j (nx+2) + i) nz + k), the order the paper's storage-order
// table compares on CPU and GPU, with the direct GPU mapping of that order:
// one thread per column (ring included), k marched inside the thread.  The
// lanes of a wavefront touch addresses nz values apart, so no load
// coalesces; this kernel exists to measure that cost.
__global__ __launch_bounds__(KIJ_BX *KIJ_BY) void k_rw_step_kij(RwArgs a) {
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int i = blockIdx.x * KIJ_BX + threadIdx.x, j = blockIdx.y * KIJ_BY + threadIdx.y;
  if (i > nx + 1 || j > ny + 1) return;
  const unsigned sj2 = unsigned(nx + 2);                 // 2D stride of j
  const unsigned si = unsigned(nz), sj = sj2 * unsigned(nz);
  const unsigned ij = unsigned(i) + unsigned(j) * sj2;
  const unsigned col = ij * si;
  const double nu = a.nu;
  if (i == 0 || i == nx + 1 || j == 0 || j == ny + 1) {
    unsigned inner, opp, iji, ijo;                       // column offsets and 2D indices
    if (i == 0 || i == nx + 1) {
      iji = i == 0 ? ij + 1 : ij - 1;
      ijo = i == 0 ? ij + unsigned(nx + 1) : ij - unsigned(nx + 1);
    } else {
      iji = j == 0 ? ij + sj2 : ij - sj2;
      ijo = j == 0 ? ij + unsigned(ny + 1) * sj2 : ij - unsigned(ny + 1) * sj2;
    }
    inner = iji * si;
    opp = ijo * si;
    for (int k = 0; k < nz; ++k) {
      const double c = phys(a, a.e[col + k], k, ij);
      const double ni = phys(a, a.e[inner + k], k, iji);
      const double no = phys(a, a.e[opp + k], k, ijo);
      a.out[col + k] = c * a.c2 + nu * (ni + no);
    }
    return;
  }
  for (int k = 0; k < nz; ++k) {
    const unsigned o = col + unsigned(k);
    const double c = phys(a, a.e[o], k, ij);
    double sum = phys(a, a.e[o - si], k, ij - 1) + phys(a, a.e[o + si], k, ij + 1);
    sum = sum + phys(a, a.e[o - sj], k, ij - sj2);
    sum = sum + phys(a, a.e[o + sj], k, ij + sj2);
    double r;
    if (k == 0) {
      sum = sum + phys(a, a.e[o + 1], 1, ij);
      r = c * a.c5 + nu * sum;
    } else if (k == nz - 1) {
      sum = sum + phys(a, a.e[o - 1], k - 1, ij);
      r = c * a.c5 + nu * sum;
    } else {
      sum = sum + phys(a, a.e[o - 1], k - 1, ij);
      sum = sum + phys(a, a.e[o + 1], k + 1, ij);
      r = c * a.c6 + nu * sum;
    }
    a.out[o] = r;
  }
}

}  // namespace

// Levels per interior block: 16, or 8 when 16-level chunks would leave fewer
// than 1024 interior blocks (four per CU), where more and shorter columns
// keep more loads in flight (128^3: 1.40 -> 1.12 ms per 100 steps; at 256^3
// and 256^2 x 512, 16 levels are 4% and 3% faster).  The cells computed do
// not depend on the chunking.
int rw_chunk(int nx, int ny, int nz, int bx, int by) {
  const long long tiles = (long long)((nx + bx - 1) / bx) * ((ny + by - 1) / by);
  const int c = tiles * ((nz + 15) / 16) < 1024 ? 8 : 16;
  return nz < c ? nz : c;
}

template <int BX, int BY>
void launch_rw_shape(RwArgs a, hipStream_t s) {
  a.tiles_x = (a.nx + BX - 1) / BX;
  a.tiles_y = (a.ny + BY - 1) / BY;
  const int ring_cells = (2 * (a.ny + 2) + 2 * a.nx) * a.nz;
  const int blocks = a.tiles_x * a.tiles_y * a.nchunk + (ring_cells + BX * BY - 1) / (BX * BY);
  hipLaunchKernelGGL((k_rw_step<BX, BY>), dim3(blocks), dim3(BX, BY), 0, s, a);
}

bool rw_block_supported(int bx, int by) {
  return (bx == 64 && by == 8) || (bx == 32 && by == 16) || (bx == 128 && by == 1) || (bx == 64 && by == 4) ||
         (bx == 128 && by == 4);
}

hipError_t launch_rw_step(const double *e, double *out, const double *surf, const double *pbl, int nx, int ny,
                          int nz, double nu, bool kij, hipStream_t s, int bx, int by) {
  RwArgs a;
  a.e = e;
  a.out = out;
  a.surf = surf;
  a.pbl = pbl;
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  a.kchunk = rw_chunk(nx, ny, nz, kij ? KIJ_BX : bx, kij ? KIJ_BY : by);
  a.tiles_x = a.tiles_y = 0;
  a.nu = nu;
  // the weights as the printed program forms them: 1 - (n nu), two roundings
  const double n6 = 6.0 * nu, n5 = 5.0 * nu, n2 = 2.0 * nu;
  a.c6 = 1.0 - n6;
  a.c5 = 1.0 - n5;
  a.c2 = 1.0 - n2;
  a.nchunk = (nz + a.kchunk - 1) / a.kchunk;
  if (kij) {
    const dim3 grid((nx + 2 + KIJ_BX - 1) / KIJ_BX, (ny + 2 + KIJ_BY - 1) / KIJ_BY);
    hipLaunchKernelGGL(k_rw_step_kij, grid, dim3(KIJ_BX, KIJ_BY), 0, s, a);
    return hipGetLastError();
  }
  if (bx == 64 && by == 8) launch_rw_shape<64, 8>(a, s);
  else if (bx == 32 && by == 16) launch_rw_shape<32, 16>(a, s);
  else if (bx == 128 && by == 1) launch_rw_shape<128, 1>(a, s);
  else if (bx == 64 && by == 4) launch_rw_shape<64, 4>(a, s);
  else if (bx == 128 && by == 4) launch_rw_shape<128, 4>(a, s);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace wx
