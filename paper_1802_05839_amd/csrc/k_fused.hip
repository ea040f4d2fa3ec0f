// Fused surrogate physics: for a tile of 128 columns, one workgroup builds the
// normalised feature rows, runs the 294-512-512-116 network on the matrix
// cores and applies the predicted theta and q tendencies to the state, so the
// activations never leave LDS (the column-local operator of the section on
// parallelisation granularity, here replaced by the learned model).
//
// Work split (8 waves, 512 threads):
//   features  thread (column = t % 128, part = t / 128); a wave covers 64
//             consecutive columns of one field level, so state reads coalesce;
//             part p forms levels [15 p, 15 p + 15) of the five profiles (part
//             3 also the surface values and the padding);
//   layers    wave w owns hidden units [64 w, 64 w + 64) of the two hidden
//             layers (2 x 4 tiles of v_mfma_f32_32x32x16_bf16, the shape that
//             runs at the full matrix-core rate on gfx950) and a 32-output by
//             64-sample block of the last; the weights are the first MFMA
//             operand (streamed from global memory in fragment order, so each
//             load is one 1 KiB run per wavefront, L2-resident, 0.98 MB, one
//             k step ahead) and the activations the second (from LDS, the
//             fragments of a k step read before its MFMAs), so a lane ends
//             with four consecutive units of one sample and stores them as
//             one 8-byte LDS write;
//   outputs   thread (column, part) updates 29 levels of theta or q with
//             coalesced read-modify-writes and the periodic halo images.
// The k order of every dot product (steps of 32 from k = 0, the same lane
// fragments) equals that of the stand-alone GEMM kernel, so both give
// bitwise-equal network outputs.
//
// LDS (133,120 B, one workgroup per CU): the input tile [128][328] BF16, the
// hidden tile [128][520] BF16 and the output tile [128][129] FP32 alias one
// buffer, with the normalisation constants of the inputs (outputs) just past
// the input (output) tile; barriers separate the phases.  Padded row strides keep the 16-byte
// fragment reads free of bank conflicts.
#include "wx_internal.h"
#include "wx_mlp_internal.h"

namespace wx {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int FT = 128;                  // columns per tile
constexpr int FTHREADS = 512;
constexpr int XLD = MLP_KIN + 8;         // 328
constexpr int HLD = MLP_NHID + 8;        // 520
constexpr int YLD = MLP_NOUTP + 1;       // 129 (FP32)
constexpr int LDS_BYTES = FT * HLD * 2;  // 133,120
static_assert(FT * XLD * 2 <= LDS_BYTES, "input tile must fit the shared buffer");
static_assert(FT * YLD * 4 <= LDS_BYTES, "output tile must fit the shared buffer");
// (mean, 1/std) of the features beside the input tile, and (mean, std) of the
// targets beside the output tile: read from LDS, the same value for a whole
// wavefront, instead of one vector load per feature and thread
constexpr int XNORM_OFF = FT * XLD * 2;
constexpr int YNORM_OFF = FT * YLD * 4;
static_assert(XNORM_OFF % 16 == 0 && XNORM_OFF + MLP_KIN * 8 <= LDS_BYTES, "feature constants must fit");
static_assert(YNORM_OFF % 16 == 0 && YNORM_OFF + MLP_NOUTP * 8 <= LDS_BYTES, "target constants must fit");
constexpr double kThetaRef = 300.0;      // theta features are theta - 300 K
constexpr int kNZ = MLP_NZ;              // levels (the network is built for 58)
constexpr int kHalf = (kNZ + 1) / 2;     // levels per thread in the update
constexpr int kPartLev = 15;             // levels per thread in the feature phase
static_assert(4 * kPartLev >= kNZ, "four parts must cover the column");

// acc[y][x] += W(units n0 + 32 y.., k) X(samples s0 + 32 x.., k) over
// k = 0..K-1 in steps of 16 (ascending, as in the stand-alone GEMM), on
// v_mfma_f32_32x32x16_bf16.  The weights are the first operand (global, in
// fragment order: the 32 x 16 block (R, S) of the [N][K] matrix is 512
// contiguous values, so a wavefront reads it as one 1 KiB run; one 32-wide k
// step fetched ahead), the activations the second (LDS [samples][lda], the
// fragments of a k step read before its MFMAs).  A lane feeds row (or column)
// lane % 32 at k = 8 (lane / 32)..+7.
template <int NU, int NS>
__device__ __forceinline__ void tile_gemm(f32x16 (&acc)[NU][NS], const uint16_t *X, int lda, int s0,
                                          const uint16_t *W, int n0, int K, int lane) {
  const int kl = 8 * (lane >> 5), rl = lane & 31;
  const int ks = K >> 4;                                  // 16-wide k blocks per row block
  const uint16_t *wp = W + (size_t)(n0 >> 5) * ks * 512 + lane * 8;
  const uint16_t *xp = X + (s0 + rl) * lda + kl;
  bf16x8 wcur[2][NU], wnext[2][NU];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int y = 0; y < NU; ++y)
      wcur[h][y] = *reinterpret_cast<const bf16x8 *>(wp + (size_t)(y * ks + h) * 512);
#pragma unroll 1
  for (int k0 = 0; k0 < K; k0 += 32) {
    const int kn = k0 + 32 < K ? k0 + 32 : k0;   // last step reloads its own slice
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int y = 0; y < NU; ++y)
        wnext[h][y] = *reinterpret_cast<const bf16x8 *>(wp + (size_t)(y * ks + (kn >> 4) + h) * 512);
    bf16x8 xf[2][NS];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int x = 0; x < NS; ++x) xf[h][x] = *reinterpret_cast<const bf16x8 *>(xp + x * 32 * lda + k0 + 16 * h);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int y = 0; y < NU; ++y)
#pragma unroll
        for (int x = 0; x < NS; ++x)
          acc[y][x] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wcur[h][y], xf[h][x], acc[y][x], 0, 0, 0);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int y = 0; y < NU; ++y) wcur[h][y] = wnext[h][y];
  }
}

// Hidden-layer epilogue: H[m][n] = bf16(relu(acc + b[n])).  Accumulator
// 4 q + c of the lane holds unit n0 + 32 y + 8 q + 4 (lane / 32) + c of sample
// 32 x + lane % 32: four consecutive BF16 values, one 8-byte LDS store.
template <int NU, int NS>
__device__ __forceinline__ void store_hidden(const f32x16 (&acc)[NU][NS], const float *b, int n0, uint16_t *H,
                                             int lane) {
#pragma unroll
  for (int y = 0; y < NU; ++y)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = n0 + 32 * y + 8 * q + 4 * (lane >> 5);
      const float4 bn = *reinterpret_cast<const float4 *>(b + n);
#pragma unroll
      for (int x = 0; x < NS; ++x) {
        const float v0 = acc[y][x][4 * q] + bn.x, v1 = acc[y][x][4 * q + 1] + bn.y;
        const float v2 = acc[y][x][4 * q + 2] + bn.z, v3 = acc[y][x][4 * q + 3] + bn.w;
        uint2 pk;
        pk.x = uint32_t(f2bf(v0 > 0.f ? v0 : 0.f)) | (uint32_t(f2bf(v1 > 0.f ? v1 : 0.f)) << 16);
        pk.y = uint32_t(f2bf(v2 > 0.f ? v2 : 0.f)) | (uint32_t(f2bf(v3 > 0.f ? v3 : 0.f)) << 16);
        *reinterpret_cast<uint2 *>(H + (32 * x + (lane & 31)) * HLD + n) = pk;
      }
    }
}

__global__ __launch_bounds__(FTHREADS) void k_surrogate_fused(FusedArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[LDS_BYTES];
  if (a.fallback && *a.fallback) return;
  const bool rows_mode = a.rows_out != nullptr;
  const int nrows = rows_mode ? (a.n_list ? min(*a.n_list, a.cap) : a.cap) : a.ncols;
  // tiles numbered so that each XCD works through a contiguous band: the
  // row above a tile (its v(j-1) reads) was loaded by a tile on the same L2
  const int r0 = xcd_remap(blockIdx.x, gridDim.x) * FT;
  if (r0 >= nrows) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nx = a.g.nx;
  uint16_t *X = reinterpret_cast<uint16_t *>(lds);
  uint16_t *H = reinterpret_cast<uint16_t *>(lds);
  float *Y = reinterpret_cast<float *>(lds);

  // ---- feature rows -> X ---------------------------------------------------
  float2 *xn = reinterpret_cast<float2 *>(lds + XNORM_OFF);
  for (int f = tid; f < MLP_KIN; f += FTHREADS) xn[f] = make_float2(a.xmean[f], a.xinvstd[f]);
  __syncthreads();
  {
    const int col = tid & (FT - 1), part = tid >> 7;
    const int r = r0 + col;
    int c = -1;
    if (r < nrows) c = rows_mode ? (a.list ? a.list[r] : r) : a.c0 + r;
    if (c >= nx * a.g.ny) c = -1;                    // not a column: zero row
    uint16_t *xr = X + col * XLD;
    auto put = [&](int f, float x) {
      const float2 mn = xn[f];
      xr[f] = f2bf((x - mn.x) * mn.y);
    };
    if (c < 0) {
      for (int f = part; f < MLP_KIN; f += 4) xr[f] = 0;
    } else {
      const int i = c % nx, j = c / nx;
      const unsigned g0 = a.g.origin + unsigned(i) + unsigned(j) * a.g.sj;
      const unsigned sk = a.g.sk, sj = a.g.sj;
      // part p builds levels [15 p, 15 p + 15) of all five profiles: it
      // first loads its levels (and the one below) into registers, so about
      // 96 independent loads are in flight, then forms the features
      const int kb = part * kPartLev, ke = min(kNZ, kb + kPartLev);
      const int k0 = kb > 0 ? kb - 1 : 0;
      float th[kPartLev + 1], qq[kPartLev + 1], ul[kPartLev + 1], uh[kPartLev + 1], vl[kPartLev + 1],
          vh[kPartLev + 1];
#pragma unroll
      for (int n = 0; n <= kPartLev; ++n) {
        const int k = k0 + n;
        if (k < ke) {
          const unsigned g = g0 + unsigned(k) * sk;
          th[n] = ldg(a.th, g);
          qq[n] = ldg(a.q, g);
          ul[n] = ldg(a.u, g - 1);
          uh[n] = ldg(a.u, g);
          vl[n] = ldg(a.v, g - sj);
          vh[n] = ldg(a.v, g);
        }
      }
      LevelVals prev{};
#pragma unroll
      for (int n = 0; n <= kPartLev; ++n) {
        const int k = k0 + n;
        if (k >= ke) break;
        LevelVals cur;
        cur.th = float(double(th[n]) + a.theta_off - kThetaRef);
        cur.q = qq[n];
        cur.u = (ul[n] + uh[n]) * 0.5f;
        cur.v = (vl[n] + vh[n]) * 0.5f;
        if (k >= kb) {
          float fv[5];
          level_features(k, cur, prev, fv);
#pragma unroll
          for (int q5 = 0; q5 < 5; ++q5) put(q5 * kNZ + k, fv[q5]);
        }
        prev = cur;
      }
      if (part == 3) {
        put(5 * kNZ, float(double(ldg(a.th_s, unsigned(c))) + a.theta_off - kThetaRef));
        put(5 * kNZ + 1, ldg(a.q_s, unsigned(c)));
        put(5 * kNZ + 2, ldg(a.f0, unsigned(c)));
        put(5 * kNZ + 3, ldg(a.ch, unsigned(c)));
        for (int f = 5 * kNZ + 4; f < MLP_KIN; ++f) xr[f] = 0;
      }
    }
  }
  __syncthreads();

  // ---- hidden layer 1: H = relu(X W1^T + b1) ---------------------------------
  f32x16 acc[2][4];
  const int n0 = wave * 64;
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[y][x][r] = 0.f;
  tile_gemm<2, 4>(acc, X, XLD, 0, a.w1, n0, MLP_KIN, lane);
  __syncthreads();   // every wave has read X
  store_hidden<2, 4>(acc, a.b1, n0, H, lane);
  __syncthreads();

  // ---- hidden layer 2: H = relu(H W2^T + b2) ---------------------------------
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[y][x][r] = 0.f;
  tile_gemm<2, 4>(acc, H, HLD, 0, a.w2, n0, MLP_NHID, lane);
  __syncthreads();
  store_hidden<2, 4>(acc, a.b2, n0, H, lane);
  __syncthreads();

  // ---- output layer: Y = H W3^T + b3 (normalised tendencies) -----------------
  // wave w: outputs [32 (w % 4), +32) of samples [64 (w / 4), +64)
  f32x16 acc3[1][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc3[0][x][r] = 0.f;
  const int o3 = 32 * (wave & 3), s3 = 64 * (wave >> 2);
  tile_gemm<1, 2>(acc3, H, HLD, s3, a.w3, o3, MLP_NHID, lane);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int o = o3 + 8 * q + 4 * (lane >> 5);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int c = 0; c < 4; ++c) Y[(s3 + 32 * x + (lane & 31)) * YLD + o + c] = acc3[0][x][4 * q + c] + a.b3[o + c];
  }
  float2 *yn = reinterpret_cast<float2 *>(lds + YNORM_OFF);
  if (!rows_mode)
    for (int o = tid; o < MLP_NOUTP; o += FTHREADS) yn[o] = make_float2(a.ymean[o], a.ystd[o]);
  __syncthreads();

  // ---- outputs ----------------------------------------------------------------
  if (rows_mode) {
    for (int e = tid; e < FT * MLP_NOUTP; e += FTHREADS) {
      const int m = e / MLP_NOUTP, o = e % MLP_NOUTP;
      if (r0 + m < nrows) a.rows_out[(size_t)(r0 + m) * MLP_NOUTP + o] = Y[m * YLD + o];
    }
    return;
  }
  const int col = tid & (FT - 1), part = tid >> 7;
  if (r0 + col >= nrows) return;
  const int c = a.c0 + r0 + col;
  if (a.judged && judge_sampled(a.seed, a.t, unsigned(c), a.rate)) return;
  const int ny = a.g.ny;
  const int i = c % nx, j = c / nx;
  const unsigned g0 = a.g.origin + unsigned(i) + unsigned(j) * a.g.sj;
  const int di = i < 2 ? nx : (i >= nx - 2 ? -nx : 0);
  const int dj = j < 2 ? ny * int(a.g.sj) : (j >= ny - 2 ? -ny * int(a.g.sj) : 0);
  float *fld = part < 2 ? a.th : a.q;
  const int kb = (part & 1) ? kHalf : 0;
  const int nk = (part & 1) ? kNZ - kHalf : kHalf;
  const int ob = (part < 2 ? 0 : kNZ) + kb;
  const float *yr = Y + col * YLD + ob;
  if (a.tend_t) {
    // tendency mode: d(theta)/dt or d(q)/dt at (i, j, k), i fastest
    float *tf = part < 2 ? a.tend_t : a.tend_q;
    for (int k = 0; k < nk; ++k) {
      const float2 ms = yn[ob + k];
      stg(tf, unsigned((kb + k) * ny + j) * unsigned(nx) + unsigned(i), fmaf(yr[k], ms.y, ms.x));
    }
    return;
  }
  const unsigned gb = g0 + unsigned(kb) * a.g.sk;
  // all loads before any store: the stores may alias the loads, so a mixed
  // order would serialise one HBM round trip per level
  float old[kHalf];
#pragma unroll
  for (int k = 0; k < kHalf; ++k)
    if (k < nk) old[k] = ldg(fld, gb + unsigned(k) * a.g.sk);
#pragma unroll
  for (int k = 0; k < kHalf; ++k) {
    if (k >= nk) break;
    const float2 ms = yn[ob + k];
    const float tend = fmaf(yr[k], ms.y, ms.x);
    const float nv = fmaf(a.dt, tend, old[k]);
    const unsigned g = gb + unsigned(k) * a.g.sk;
    stg(fld, g, nv);
    if (di != 0) stg(fld, g + di, nv);
    if (dj != 0) {
      stg(fld, g + dj, nv);
      if (di != 0) stg(fld, g + dj + di, nv);
    }
  }
}

}  // namespace

hipError_t launch_surrogate_fused(const FusedArgs &a, hipStream_t s) {
  const int rows = a.rows_out ? a.cap : a.ncols;
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_surrogate_fused, dim3((rows + FT - 1) / FT), dim3(FTHREADS), 0, s, a);
  return hipGetLastError();
}

}  // namespace wx
