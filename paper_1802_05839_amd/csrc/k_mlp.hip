// The learned surrogate of the column physics: BF16 MFMA GEMMs with FP32
// accumulation, loss, Adam, initialisation, feature/label assembly and
// normalisation.
//
// Method (readings; the paper has no learned component): a 294-512-512-116
// ReLU network maps a column's physics inputs to its theta and q tendencies;
// GEMM operands (inputs, activations, weights, upstream gradients) are BF16
// rounded to nearest even, accumulation is FP32, bias / ReLU / loss / bias
// gradients / Adam are FP32; weights are stored FP32 (master) with BF16
// copies refreshed after each update.
//
// GEMM: C[m][n] = sum_k A(m,k) B(k,n) on 64 x 64 output tiles, K staged in
// steps of 32, four waves each owning a 32 x 32 quarter as one tile of
// v_mfma_f32_32x32x16_bf16 (two instructions per 32-wide k step, k ascending;
// on gfx950 this shape runs at twice the rate of the 16x16x32 one).  Operands
// are staged through LDS in [row][k] order (k contiguous) so each lane feeds
// the matrix core with one 16-byte LDS read per operand and instruction;
// global operands may be k-contiguous (row-major [rows][K]) or row-contiguous
// ([K][rows]); the latter are transposed on the way into LDS (with a chunk
// swizzle against bank conflicts).  Each thread's 16-byte operand chunks
// travel four k steps ahead in registers, so a step's global round trip
// overlaps the matrix work of the steps before it.  Two independent GEMMs
// (a weight gradient and the hidden gradient reading the same delta) can
// share one launch.
// Every output element is produced by one lane with a fixed k order, and a
// split over K writes partial tiles that a second kernel sums in a fixed order,
// so results are bitwise reproducible.
#include <type_traits>

#include "wx_internal.h"
#include "wx_mlp_internal.h"

namespace wx {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int GBM = 64, GBN = 64, GBK = 32, GLD = GBK + 8;  // LDS row stride (bf16 elements)
constexpr int GPF = 4;      // k steps whose operand chunks are in flight beyond the one in LDS (even)
constexpr int GKIDX = 256;  // longest k range per block whose k rows may be gathered

// Staging of one 64 x 32 operand tile (rows r0.., k k0..) into LDS as
// [row][k], split into its global half (this thread's 16-byte chunk, loaded
// a few k steps ahead into registers) and its LDS half.
// KCONTIG: memory is [rows][ld] with k contiguous; the thread owns tile row
// t / 4 (memory row grow: the batch gather resolved once per block, -1 past
// the operand) at k = k0 + 8 (t % 4).  Otherwise memory is [K][ld] with rows
// contiguous; the thread owns k row k0 + t / 8 (memory row kidx[k - kb] when
// the k rows are gathered, from the block's index table in LDS) at tile rows
// 8 (t % 8)..+7, transposed on the way into LDS.  In a transposed tile the
// four 8-wide k chunks of row r sit in the order chunk ^ ((r / 8) % 4): the
// eight rows a thread writes are 8 apart, which with any 16-byte-aligned row
// stride falls on one LDS bank, and the swizzle spreads them over four.
__device__ __forceinline__ int tile_slot(int r, int k, bool swz) {
  return r * GLD + (swz ? ((((k >> 3) ^ (r >> 3)) & 3) << 3) + (k & 7) : k);
}
template <bool KCONTIG>
__device__ __forceinline__ uint4 chunk_load(const uint16_t *g, int ld, int r0, int k0, int nrows, int nk, int grow,
                                            const int *kidx, int kb) {
  const int t = threadIdx.x;
  uint4 v = make_uint4(0, 0, 0, 0);
  if (KCONTIG) {
    const int gk = k0 + (t & 3) * 8;
    if (grow >= 0 && gk < nk) v = *reinterpret_cast<const uint4 *>(g + (size_t)grow * ld + gk);
  } else {
    const int gk = k0 + (t >> 3), gr = r0 + (t & 7) * 8;
    if (gk < nk && gr < nrows) {
      const int krow = kidx ? kidx[gk - kb] : gk;
      v = *reinterpret_cast<const uint4 *>(g + (size_t)krow * ld + gr);
    }
  }
  return v;
}

template <bool KCONTIG>
__device__ __forceinline__ void chunk_store(uint16_t *lds, const uint4 &v) {
  const int t = threadIdx.x;
  if (KCONTIG) {
    *reinterpret_cast<uint4 *>(lds + (t >> 2) * GLD + (t & 3) * 8) = v;
  } else {
    const int kk = t >> 3, r = (t & 7) * 8;
    uint16_t *dst = lds + tile_slot(r, kk, true);   // rows r..r+7 share the chunk order
    const uint16_t *e = reinterpret_cast<const uint16_t *>(&v);
#pragma unroll
    for (int q = 0; q < 8; ++q) dst[q * GLD] = e[q];
  }
}

// Epilogue kinds
enum { EP_F32 = 0, EP_BIAS_F32 = 1, EP_BIAS_RELU_BF16 = 2, EP_PARTIAL_F32 = 4, EP_MASK_F32_BF16 = 5 };

struct GemmArgs {
  const uint16_t *A, *B;
  int lda, ldb;
  int M, N, K;                 // logical sizes (K = reduction length of this launch's split)
  int k_split;                 // K elements per split (grid.z splits)
  const int *rows_a;           // optional gather of A's rows (KCONTIG) or k rows (not KCONTIG)
  const int *rows_b;           // optional gather of B's k rows (B not KCONTIG)
  const float *bias;           // [N]
  void *C;                     // output
  int ldc;
  size_t split_stride;         // EP_PARTIAL_F32: elements between split slices
  const uint16_t *mask;        // EP_MASK_F32_BF16: BF16 activation, C's layout
  uint16_t *C2;                // EP_MASK_F32_BF16: BF16 copy of the output
  float *colpart;              // EP_MASK_F32_BF16, optional: [M / 32][ldc] column sums of 32-row groups
};

// Tile (m0, n0, split) of linear block lin of a GEMM whose grid is nbn x nbm
// x nbz (n tiles, m tiles, K splits).  Blocks are dealt round-robin to the 8
// XCDs; the remap gives each XCD a contiguous run of the linear order (n
// fastest, then m, then the split), so an XCD's blocks share their A rows and
// K range in its L2 and the blocks running together spread over all n tiles.
struct GemmTile {
  int m0, n0, z;
};
__device__ __forceinline__ GemmTile gemm_tile(int lin, int nbn, int nbm, int nbz) {
  const int L = xcd_remap(lin, nbn * nbm * nbz);
  GemmTile t;
  t.n0 = (L % nbn) * GBN;
  t.m0 = ((L / nbn) % nbm) * GBM;
  t.z = L / (nbn * nbm);
  return t;
}

// Output of one wave's 32 x 32 tile (origin m0 + wm, n0 + wn).
template <int EP>
__device__ __forceinline__ void gemm_epilogue(const GemmArgs &a, const f32x16 &acc, int m0, int n0, int z, int wm,
                                              int wn, int lane) {
  // accumulator r of the lane holds C[8 (r / 4) + 4 (lane / 32) + r % 4][lane % 32]
  // of the wave's 32 x 32 tile.  Everything the lane reads (its column's bias,
  // the masks of its 16 rows) is read before its first store: a read after a
  // store that may alias it would wait for a full memory round trip per row.
  const int n = n0 + wn + (lane & 31);
  const bool nok = n < a.N;
  float bias = 0.f;
  if ((EP == EP_BIAS_F32 || EP == EP_BIAS_RELU_BF16) && nok) bias = a.bias[n];
  uint16_t mk[16];
  if (EP == EP_MASK_F32_BF16) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      mk[r] = (m < a.M && nok) ? a.mask[(size_t)m * a.ldc + n] : uint16_t(0);
    }
  }
  auto emit = [&](int r, int m) {
    float v = acc[r];
    if (EP == EP_F32) {
      static_cast<float *>(a.C)[(size_t)m * a.ldc + n] = v;
    } else if (EP == EP_BIAS_F32) {
      static_cast<float *>(a.C)[(size_t)m * a.ldc + n] = v + bias;
    } else if (EP == EP_BIAS_RELU_BF16) {
      v += bias;
      static_cast<uint16_t *>(a.C)[(size_t)m * a.ldc + n] = f2bf(v > 0.f ? v : 0.f);
    } else if (EP == EP_MASK_F32_BF16) {
      // hidden-layer gradient: (upstream @ W) * (h > 0), FP32 and its BF16 operand
      const size_t o = (size_t)m * a.ldc + n;
      const float g = bf2f(mk[r]) > 0.f ? v : 0.f;
      static_cast<float *>(a.C)[o] = g;
      a.C2[o] = f2bf(g);
    } else {
      static_cast<float *>(a.C)[z * a.split_stride + (size_t)m * a.ldc + n] = v;
    }
  };
  if (EP == EP_MASK_F32_BF16 && a.colpart) {
    // the wave's 32 rows of column n summed: the lane's 16 rows in r order
    // (rows past M and masked entries are 0), then the half-wave holding rows
    // 8 q + 0..3 plus the one holding rows 8 q + 4..7; the bias gradient is
    // then a sum over M / 32 of these instead of M rows
    float p = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      p += (m < a.M && nok && bf2f(mk[r]) > 0.f) ? acc[r] : 0.f;
    }
    const float o = __shfl_xor(p, 32);
    const float t = lane < 32 ? p + o : o + p;
    // a wave whose 32 rows all lie past M has no group (the buffer holds ceil(M / 32))
    if (lane < 32 && nok && m0 + wm < a.M) a.colpart[(size_t)((m0 + wm) >> 5) * a.ldc + n] = t;
  }
  // a wave whose 32 x 32 tile lies inside C stores with no per-row test:
  // divergent per-row branches would make every store wait for the one
  // before it (the vector-memory counter also counts stores)
  if (m0 + wm + 32 <= a.M && n0 + wn + 32 <= a.N) {
#pragma unroll
    for (int r = 0; r < 16; ++r) emit(r, m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3));
  } else {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = m0 + wm + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (m < a.M && nok) emit(r, m);
    }
  }
}

// LDS of one GEMM block: the two staged k steps of both operands and the k
// gather tables.
struct GemmLds {
  uint16_t sA[2][GBM * GLD];
  uint16_t sB[2][GBN * GLD];
  int ka[GKIDX], kb[GKIDX];
};

// One 64 x 64 output tile: linear block lin of a GEMM with an nbn x nbm x
// nbz grid.
template <bool AK, bool BK_, int EP>
__device__ __forceinline__ void gemm_block(const GemmArgs &a, GemmLds &lds, int lin, int nbn, int nbm, int nbz) {
  uint16_t (&sA)[2][GBM * GLD] = lds.sA;
  uint16_t (&sB)[2][GBN * GLD] = lds.sB;
  int *s_ka = lds.ka, *s_kb = lds.kb;
  const GemmTile tile = gemm_tile(lin, nbn, nbm, nbz);
  const int m0 = tile.m0, n0 = tile.n0;
  const int kb = tile.z * a.k_split;
  const int ke = min(a.K, kb + a.k_split);
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;

  // the gathers, resolved before the k loop: a k-contiguous operand's row
  // per thread, a row-contiguous operand's k rows into an LDS table
  const int *ka = nullptr, *kbt = nullptr;
  int growa = -1, growb = -1;
  if (AK) {
    const int gr = m0 + (t >> 2);
    if (gr < a.M) growa = a.rows_a ? a.rows_a[gr] : gr;
  } else if (a.rows_a) {
    for (int q = t; q < ke - kb; q += 256) s_ka[q] = a.rows_a[kb + q];
    ka = s_ka;
  }
  if (BK_) {
    const int gr = n0 + (t >> 2);
    if (gr < a.N) growb = a.rows_b ? a.rows_b[gr] : gr;
  } else if (a.rows_b) {
    for (int q = t; q < ke - kb; q += 256) s_kb[q] = a.rows_b[kb + q];
    kbt = s_kb;
  }
  __syncthreads();

  // k step s is staged in LDS buffer s & 1; the chunks of the next GPF steps
  // are in flight in register slots (step s in slot s % GPF), so the global
  // round trip of a step overlaps the matrix work of the GPF steps before it
  const int nsteps = (ke - kb + GBK - 1) / GBK;
  uint4 pa[GPF], pb[GPF];
  auto fetch = [&](int s, int slot) {
    const int k0 = kb + s * GBK;
    pa[slot] = chunk_load<AK>(a.A, a.lda, m0, k0, a.M, ke, growa, ka, kb);
    pb[slot] = chunk_load<BK_>(a.B, a.ldb, n0, k0, a.N, ke, growb, kbt, kb);
  };
#pragma unroll
  for (int d = 0; d < GPF; ++d)
    if (d < nsteps) fetch(d, d);
  if (nsteps > 0) {
    chunk_store<AK>(sA[0], pa[0]);
    chunk_store<BK_>(sB[0], pb[0]);
    if (GPF < nsteps) fetch(GPF, 0);
  }
  __syncthreads();
  // lane holds row (or column) lane % 32 of its operand at k = 8 (lane / 32)..+7
  // of each 16-wide half of a step (transposed tiles: swizzled chunks)
  const int ra0 = tile_slot(wm + (lane & 31), 8 * (lane >> 5), !AK);
  const int ra1 = tile_slot(wm + (lane & 31), 16 + 8 * (lane >> 5), !AK);
  const int rb0 = tile_slot(wn + (lane & 31), 8 * (lane >> 5), !BK_);
  const int rb1 = tile_slot(wn + (lane & 31), 16 + 8 * (lane >> 5), !BK_);
  // step s with c = s % GPF a compile-time constant, so that every register
  // slot and LDS buffer is fixed
  auto step = [&](int s, auto cc) __attribute__((always_inline)) {
    constexpr int c = decltype(cc)::value;
    constexpr int buf = c & 1, nslot = (c + 1) % GPF;
    static_assert(GBK == 32, "two 16-wide halves per step");
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const bf16x8 fa = *reinterpret_cast<const bf16x8 *>(sA[buf] + (h ? ra1 : ra0));
      const bf16x8 fb = *reinterpret_cast<const bf16x8 *>(sB[buf] + (h ? rb1 : rb0));
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa, fb, acc, 0, 0, 0);
    }
    if (s + 1 < nsteps) {
      // buffer buf ^ 1 was last read in step s - 1, which every wave has left
      chunk_store<AK>(sA[buf ^ 1], pa[nslot]);
      chunk_store<BK_>(sB[buf ^ 1], pb[nslot]);
      if (s + 1 + GPF < nsteps) fetch(s + 1 + GPF, nslot);
    }
    __syncthreads();
  };
  static_assert(GPF == 4, "the loop below is unrolled for four slots");
  for (int s0 = 0; s0 < nsteps; s0 += GPF) {
    step(s0, std::integral_constant<int, 0>());
    if (s0 + 1 < nsteps) step(s0 + 1, std::integral_constant<int, 1>());
    if (s0 + 2 < nsteps) step(s0 + 2, std::integral_constant<int, 2>());
    if (s0 + 3 < nsteps) step(s0 + 3, std::integral_constant<int, 3>());
  }
  gemm_epilogue<EP>(a, acc, m0, n0, tile.z, wm, wn, lane);
}

template <bool AK, bool BK_, int EP>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs a) {
  __shared__ __attribute__((aligned(16))) GemmLds lds;
  gemm_block<AK, BK_, EP>(a, lds, blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), gridDim.x,
                          gridDim.y, gridDim.z);
}

// Two independent GEMMs in one launch (the weight gradient and the input
// gradient that read the same upstream delta): blocks [0, n1) are the first
// GEMM's, [n1p, n1p + n2) the second's, n1p = n1 rounded up to a multiple of 8
// so that each GEMM's blocks keep their XCD order (the blocks in between
// return at once).  Each block computes exactly what it would in a launch of
// its own; the smaller GEMM runs in the larger one's shadow instead of after
// it.
struct GemmGrid {
  int nbn, nbm, nbz;
};
template <bool AK1, bool BK1, int EP1, bool AK2, bool BK2, int EP2>
__global__ __launch_bounds__(256) void k_gemm_pair(GemmArgs a1, GemmGrid g1, GemmArgs a2, GemmGrid g2, int n1p) {
  __shared__ __attribute__((aligned(16))) GemmLds lds;
  const int b = blockIdx.x;
  if (b < n1p) {
    if (b < g1.nbn * g1.nbm * g1.nbz) gemm_block<AK1, BK1, EP1>(a1, lds, b, g1.nbn, g1.nbm, g1.nbz);
  } else {
    gemm_block<AK2, BK2, EP2>(a2, lds, b - n1p, g2.nbn, g2.nbm, g2.nbz);
  }
}

// Loss and output gradient: d = 2 (y - t) / (B * nout) on the first nout
// outputs (0 on padding), as FP32 and BF16; per-row partial loss sums.
__global__ __launch_bounds__(256) void k_loss(const float *y, const float *t, const int *rows, int batch, int nout,
                                              int ldy, float *d32, uint16_t *d16, float *row_loss) {
  // a wave per batch row; lane l holds outputs l and l + 64 of the 128 padded
  const int lane = threadIdx.x & 63;
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= batch) return;                           // whole waves
  const int row = rows ? rows[m] : m;
  float sq[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int n = lane + 64 * h;
    float e = 0.f, g = 0.f;
    if (n < nout) {
      e = y[(size_t)m * ldy + n] - t[(size_t)row * ldy + n];
      g = 2.f * e / float(batch * nout);
    }
    d32[(size_t)m * ldy + n] = g;
    d16[(size_t)m * ldy + n] = f2bf(g);
    sq[h] = settle(e * e);
  }
  // the row's sum of squares by halving: (n, n + 64), then (n, n + 32), ...
  // down to lane 0, each partial a rounded FP32 sum
  float v = sq[0] + sq[1];
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) v = settle(v + __shfl_down(v, w));
  if (lane == 0) row_loss[m] = v;
}

// One Adam update of element i of tensor S with gradient g; refreshes the
// BF16 copies (row-major, transposed, fragment order) that exist.
__device__ __forceinline__ void adam_elem(const AdamArgs &a, const AdamSeg &S, size_t i, float g) {
  const float mi = 0.9f * S.m[i] + 0.1f * g;
  const float vi = 0.999f * S.v[i] + 0.001f * g * g;
  S.m[i] = mi;
  S.v[i] = vi;
  const float wi = S.w[i] - a.lr * (mi / a.bc1) / (sqrtf(vi / a.bc2) + 1e-8f);
  S.w[i] = wi;
  if (S.wb) {
    const uint16_t h = f2bf(wi);
    S.wb[i] = h;
    const int r = int(i / S.cols), c = int(i % S.cols);
    if (S.wbt) S.wbt[(size_t)c * S.rows + r] = h;
    if (S.wbp) S.wbp[frag_index(r, c, S.cols)] = h;
  }
}

// Column sums of up to four [rows][lda] FP32 matrices (one block's share).
// Block b covers COLSUM_COLS = 16 columns of one matrix; thread (quad q,
// group g) sums columns 16b + 4q .. 16b + 4q + 3 over rows g, g + 64, ... in
// order (float4 loads when the matrix allows, sixteen rows in flight
// together), then the 64 group sums are folded in a fixed tree.  These
// blocks run on few CUs, so their speed is the bytes each keeps in flight.
__device__ __forceinline__ void colsum_block(const ColsumArgs &a, int b, const AdamArgs *adam, const int *seg) {
  static_assert(COLSUM_COLS == 16, "four float4 quads of columns per block");
  __shared__ float sh[64][17];
  int jb = 0;
  while (jb + 1 < a.njobs && b >= a.job[jb].blocks) {
    b -= a.job[jb].blocks;
    ++jb;
  }
  const ColsumJob &J = a.job[jb];
  const int rows = J.rows > 0 ? J.rows : a.rows;
  const int q = threadIdx.x & 3, g = threadIdx.x >> 2;
  const int c = b * 16 + 4 * q;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  if (J.vec) {
    if (c < J.cols) {
      int r = g;
      for (; r + 15 * 64 < rows; r += 16 * 64) {
        float4 x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) x[u] = *reinterpret_cast<const float4 *>(J.a + (size_t)(r + 64 * u) * J.lda + c);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          s0 += x[u].x;
          s1 += x[u].y;
          s2 += x[u].z;
          s3 += x[u].w;
        }
      }
      for (; r < rows; r += 64) {
        const float4 x = *reinterpret_cast<const float4 *>(J.a + (size_t)r * J.lda + c);
        s0 += x.x;
        s1 += x.y;
        s2 += x.z;
        s3 += x.w;
      }
    }
  } else {
    // scalar loads (the loss column): also sixteen rows in flight; a loop
    // with one load per row would wait a full round trip per row
    const int nc = min(4, J.cols - c);
    int r = g;
    for (; r + 15 * 64 < rows; r += 16 * 64) {
      float x[16][4];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const float *row = J.a + (size_t)(r + 64 * u) * J.lda + c;
#pragma unroll
        for (int e = 0; e < 4; ++e) x[u][e] = e < nc ? row[e] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        s0 += x[u][0];
        s1 += x[u][1];
        s2 += x[u][2];
        s3 += x[u][3];
      }
    }
    for (; r < rows; r += 64) {
      const float *row = J.a + (size_t)r * J.lda + c;
      if (nc > 0) s0 += row[0];
      if (nc > 1) s1 += row[1];
      if (nc > 2) s2 += row[2];
      if (nc > 3) s3 += row[3];
    }
  }
  sh[g][4 * q] = s0;
  sh[g][4 * q + 1] = s1;
  sh[g][4 * q + 2] = s2;
  sh[g][4 * q + 3] = s3;
  __syncthreads();
  const int col = threadIdx.x & 15, grp = threadIdx.x >> 4;   // 16 columns x 16 lanes
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1) {
    for (int gg = grp; gg < h; gg += 16) sh[gg][col] += sh[gg + h][col];
    __syncthreads();
  }
  if (threadIdx.x < 16 && b * 16 + col < J.cols) {
    J.out[b * 16 + col] = sh[0][col];
    if (adam && seg[jb] >= 0) adam_elem(*adam, adam->seg[seg[jb]], size_t(b * 16 + col), sh[0][col]);
  }
}

// The bias-gradient and loss column sums (first blocks: each sums all batch
// rows of 16 columns, the longest blocks of the launch, so they start first),
// then the weight gradients as ordered sums of split-K slices; with adam_on
// each gradient element also takes its Adam update right where it is formed.
__global__ void __launch_bounds__(256) k_grad_finish(GradFinishArgs a) {
  int b = blockIdx.x;
  int csb = 0;
  for (int j = 0; j < a.cs.njobs; ++j) csb += a.cs.job[j].blocks;
  if (b < csb) {
    colsum_block(a.cs, b, a.adam_on ? &a.adam : nullptr, a.cs_seg);
    return;
  }
  b -= csb;
  for (int j = 0; j < a.nsj; ++j) {
    const SplitJob &J = a.sj[j];
    if (b < J.blocks) {
      const int i = b * 256 + threadIdx.x;
      if (i >= J.n) return;
      // slices in batches of 16 loads in flight, summed in slice order
      float s = 0.f;
      int p = 0;
      for (; p + 16 <= J.nsplit; p += 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = J.part[(p + u) * J.stride + i];
#pragma unroll
        for (int u = 0; u < 16; ++u) s += v[u];
      }
      for (; p < J.nsplit; ++p) s += J.part[p * J.stride + i];
      J.out[i] = s;
      if (a.adam_on) adam_elem(a.adam, a.adam.seg[a.sj_seg[j]], size_t(i), s);
      return;
    }
    b -= J.blocks;
  }
}

// Adam over the six parameter tensors in one launch (element i of the
// concatenation belongs to the tensor whose range holds it).
__global__ void k_adam_multi(AdamArgs a) {
  const size_t gi = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  int t = 0;
  while (t + 1 < 6 && gi >= a.seg[t + 1].start) ++t;
  const AdamSeg &S = a.seg[t];
  const size_t i = gi - S.start;
  if (i >= S.n) return;
  adam_elem(a, S, i, S.g[i]);
}

// BF16 copies of FP32 weights (after initialisation or an upload).
__global__ void k_to_bf16(const float *w, size_t n, uint16_t *wb, uint16_t *wbt, uint16_t *wbp, int rows,
                          int cols) {
  const size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint16_t h = f2bf(w[i]);
  wb[i] = h;
  const int r = int(i / cols), c = int(i % cols);
  if (wbt) wbt[(size_t)c * rows + r] = h;
  if (wbp) wbp[frag_index(r, c, cols)] = h;
}


// He-uniform init of a (fan_out x fan_in) block inside a padded (rows x ld)
// FP32 matrix; element e = r * fan_in + c draws SplitMix64 of
// (seed << 32) | (tensor << 28) | e.
__global__ void k_he_init(float *w, int ld, int fan_out, int fan_in, uint64_t seed, int tensor, float bound) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= fan_out * fan_in) return;
  const int r = e / fan_in, c = e % fan_in;
  const uint64_t z = splitmix64((seed << 32) | (uint64_t(tensor) << 28) | uint64_t(e));
  const float u = float(uint32_t(z >> 40)) * (1.0f / 16777216.0f);
  w[(size_t)r * ld + c] = (2.0f * u - 1.0f) * bound;
}

// Epoch shuffle: element i of a Feistel permutation of [0, 2^(2h)) (four
// rounds, SplitMix64 round function keyed by seed, epoch and round), applied
// again while the value is >= n (cycle walking keeps it a permutation of
// [0, n)).
__device__ __forceinline__ uint32_t feistel(uint32_t x, int h, uint64_t key) {
  const uint32_t mask = (1u << h) - 1u;
  uint32_t l = x >> h, r = x & mask;
#pragma unroll
  for (int round = 0; round < 4; ++round) {
    const uint32_t f = uint32_t(splitmix64(key ^ (uint64_t(round) << 56) ^ uint64_t(r))) & mask;
    const uint32_t nl = r, nr = l ^ f;
    l = nl;
    r = nr;
  }
  return (l << h) | r;
}

__global__ void k_shuffle(uint64_t key, int h, int n, int m, int32_t *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  uint32_t x = uint32_t(i);
  do {
    x = feistel(x, h, key);
  } while (x >= uint32_t(n));
  out[i] = int32_t(x);
}

}  // namespace

// Kernel arguments and grid of a GEMM; false if the spec is not supported.
static bool gemm_setup(const GemmSpec &g, GemmArgs &a, GemmGrid &grid) {
  a.A = g.A; a.B = g.B; a.lda = g.lda; a.ldb = g.ldb;
  a.M = g.M; a.N = g.N; a.K = g.K;
  a.k_split = g.splits > 1 ? (g.K + g.splits - 1) / g.splits : g.K;
  a.k_split = (a.k_split + GBK - 1) / GBK * GBK;
  a.rows_a = g.rows_a; a.rows_b = g.rows_b; a.bias = g.bias;
  a.C = g.C; a.ldc = g.ldc; a.split_stride = g.split_stride;
  a.mask = g.mask; a.C2 = g.C2; a.colpart = g.colpart;
  const int splits = g.splits > 1 ? (g.K + a.k_split - 1) / a.k_split : 1;
  // a gather over k goes through a per-block index table of GKIDX entries
  if (((!g.a_kcontig && g.rows_a) || (!g.b_kcontig && g.rows_b)) && a.k_split > GKIDX) return false;
  if (g.epilogue == GEMM_MASK_F32_BF16 && (!g.mask || !g.C2)) return false;
  grid = {(g.N + GBN - 1) / GBN, (g.M + GBM - 1) / GBM, splits};
  const int key = (g.a_kcontig ? 1 : 0) | (g.b_kcontig ? 2 : 0);
  return g.epilogue == GEMM_PARTIAL_F32 ? key == 0 : key == 3;
}

hipError_t launch_gemm(const GemmSpec &g, hipStream_t s) {
  GemmArgs a;
  GemmGrid gg;
  if (!gemm_setup(g, a, gg)) return hipErrorInvalidValue;
  const dim3 grid(gg.nbn, gg.nbm, gg.nbz);
#define WX_G(AK, BK, EP) hipLaunchKernelGGL((k_gemm<AK, BK, EP>), grid, dim3(256), 0, s, a)
  switch (g.epilogue) {
    case GEMM_BIAS_RELU_BF16: WX_G(true, true, EP_BIAS_RELU_BF16); break;
    case GEMM_BIAS_F32: WX_G(true, true, EP_BIAS_F32); break;
    case GEMM_F32: WX_G(true, true, EP_F32); break;
    case GEMM_MASK_F32_BF16: WX_G(true, true, EP_MASK_F32_BF16); break;
    case GEMM_PARTIAL_F32: WX_G(false, false, EP_PARTIAL_F32); break;
    default: return hipErrorInvalidValue;
  }
#undef WX_G
  return hipGetLastError();
}

hipError_t launch_gemm_pair(const GemmSpec &g1, const GemmSpec &g2, hipStream_t s) {
  if (g1.epilogue != GEMM_PARTIAL_F32 || g2.epilogue != GEMM_MASK_F32_BF16) return hipErrorInvalidValue;
  GemmArgs a1, a2;
  GemmGrid gg1, gg2;
  if (!gemm_setup(g1, a1, gg1) || !gemm_setup(g2, a2, gg2)) return hipErrorInvalidValue;
  const int n1 = gg1.nbn * gg1.nbm * gg1.nbz, n2 = gg2.nbn * gg2.nbm * gg2.nbz;
  const int n1p = (n1 + 7) / 8 * 8;
  hipLaunchKernelGGL((k_gemm_pair<false, false, EP_PARTIAL_F32, true, true, EP_MASK_F32_BF16>), dim3(n1p + n2),
                     dim3(256), 0, s, a1, gg1, a2, gg2, n1p);
  return hipGetLastError();
}

hipError_t launch_loss(const float *y, const float *t, const int *rows, int batch, int nout, int ldy,
                       float *d32, uint16_t *d16, float *row_loss, hipStream_t s) {
  if (nout > 128) return hipErrorInvalidValue;       // a wave covers 128 padded outputs
  hipLaunchKernelGGL(k_loss, dim3((batch + 3) / 4), dim3(256), 0, s, y, t, rows, batch, nout, ldy, d32, d16, row_loss);
  return hipGetLastError();
}

hipError_t launch_shuffle(uint64_t seed, uint64_t epoch, int n, int m, int32_t *out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  int h = 1;
  while ((1ll << (2 * h)) < (long long)n) ++h;
  const uint64_t key = splitmix64(seed) ^ splitmix64(epoch ^ 0x5851F42D4C957F2Dull);
  hipLaunchKernelGGL(k_shuffle, dim3((m + 255) / 256), dim3(256), 0, s, key, h, n, m, out);
  return hipGetLastError();
}

hipError_t launch_grad_finish(const GradFinishArgs &a, hipStream_t s) {
  int blocks = 0;
  for (int j = 0; j < a.nsj; ++j) blocks += a.sj[j].blocks;
  for (int j = 0; j < a.cs.njobs; ++j) blocks += a.cs.job[j].blocks;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_finish, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_adam_multi(const AdamArgs &a, hipStream_t s) {
  const size_t n = a.seg[5].start + a.seg[5].n;
  hipLaunchKernelGGL(k_adam_multi, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float *w, size_t n, uint16_t *wb, uint16_t *wbt, uint16_t *wbp, int rows, int cols,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, w, n, wb, wbt, wbp, rows, cols);
  return hipGetLastError();
}

hipError_t launch_he_init(float *w, int ld, int fan_out, int fan_in, uint64_t seed, int tensor, float bound,
                          hipStream_t s) {
  const int n = fan_out * fan_in;
  hipLaunchKernelGGL(k_he_init, dim3((n + 255) / 256), dim3(256), 0, s, w, ld, fan_out, fan_in, seed, tensor, bound);
  return hipGetLastError();
}

}  // namespace wx
