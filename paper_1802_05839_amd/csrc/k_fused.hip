// Fused surrogate physics: for a tile of 128 columns, one workgroup builds the
// normalised feature rows, runs the 294-512-512-116 network on the matrix
// cores and applies the predicted theta and q tendencies to the state, so the
// activations never leave LDS (the column-local operator of the section on
// parallelisation granularity, here replaced by the learned model).
//
// Work split (8 waves, 512 threads):
//   features  thread (column = t % 128, part = t / 128); a wave covers 64
//             consecutive columns of one field level, so state reads coalesce;
//             part p forms levels [16 p, 16 p + 16) of the five profiles (part
//             3 also the surface values and the padding), two features per
//             4-byte LDS store;
//   layers    wave w owns hidden units [64 w, 64 w + 64) of the two hidden
//             layers (2 x 4 tiles of v_mfma_f32_32x32x16_bf16, the shape that
//             runs at the full matrix-core rate on gfx950) and a 32-output by
//             64-sample block of the last; the weights are the first MFMA
//             operand (streamed from global memory in fragment order, so each
//             load is one 1 KiB run per wavefront, L2-resident, 0.98 MB, two
//             k steps ahead) and the activations the second (from LDS, the
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
constexpr int kPartLev = 16;             // levels per thread in the feature phase (even: features go in pairs)
static_assert(4 * kPartLev >= kNZ, "four parts must cover the column");

// acc[y][x] += W(units n0 + 32 y.., k) X(samples s0 + 32 x.., k) over
// k = 0..K-1 in steps of 16 (ascending, as in the stand-alone GEMM), on
// v_mfma_f32_32x32x16_bf16.  The weights are the first operand (global, in
// fragment order: the 32 x 16 block (R, S) of the [N][K] matrix is 512
// contiguous values, so a wavefront reads it as one 1 KiB run; fetched two
// 32-wide k steps ahead, so an L2 round trip overlaps two steps of MFMAs),
// the activations the second (LDS [samples][lda], the
// fragments of a k step read before its MFMAs).  A lane feeds row (or column)
// lane % 32 at k = 8 (lane / 32)..+7.
template <int NU, int NS, int K>
__device__ __forceinline__ void tile_gemm(f32x16 (&acc)[NU][NS], const uint16_t *X, int lda, int s0,
                                          const uint16_t *W, int n0, int lane) {
  constexpr int ks = K >> 4;                              // 16-wide k blocks per row block
  constexpr int NSTEP = K / 32;                           // 32-wide k steps
  constexpr int D = 2;                                    // steps the weights are fetched ahead
  static_assert(K % 32 == 0, "K must be a multiple of 32");
  const int kl = 8 * (lane >> 5), rl = lane & 31;
  const uint16_t *wp = W + (size_t)(n0 >> 5) * ks * 512 + lane * 8;
  const uint16_t *xp = X + (s0 + rl) * lda + kl;
  bf16x8 wr[D + 1][2][NU];
  auto wload = [&](int s) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int y = 0; y < NU; ++y)
        wr[s % (D + 1)][h][y] = *reinterpret_cast<const bf16x8 *>(wp + (size_t)(y * ks + 2 * s + h) * 512);
  };
#pragma unroll
  for (int s = 0; s < D; ++s)
    if (s < NSTEP) wload(s);
#pragma unroll
  for (int s = 0; s < NSTEP; ++s) {
    if (s + D < NSTEP) wload(s + D);
    bf16x8 xf[2][NS];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int x = 0; x < NS; ++x) xf[h][x] = *reinterpret_cast<const bf16x8 *>(xp + x * 32 * lda + 32 * s + 16 * h);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int y = 0; y < NU; ++y)
#pragma unroll
        for (int x = 0; x < NS; ++x)
          acc[y][x] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wr[s % (D + 1)][h][y], xf[h][x], acc[y][x], 0, 0, 0);
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
        pk.x = f2bf2(v0 > 0.f ? v0 : 0.f, v1 > 0.f ? v1 : 0.f);
        pk.y = f2bf2(v2 > 0.f ? v2 : 0.f, v3 > 0.f ? v3 : 0.f);
        *reinterpret_cast<uint2 *>(H + (32 * x + (lane & 31)) * HLD + n) = pk;
      }
    }
}

__global__ __launch_bounds__(FTHREADS) void k_surrogate_fused(FusedArgs a) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[LDS_BYTES];
  // the three bias vectors, staged with the feature loads: read from LDS in
  // the layer epilogues, they never wait behind a global round trip
  __shared__ __attribute__((aligned(16))) float s_bias[2 * MLP_NHID + MLP_NOUTP];
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
  // thread (column = t % 128, part = t / 128); part p builds levels
  // [16 p, 16 p + 16) of the five profiles (part 3 also the surface values
  // and the padding).  Its loads (its levels and the one below, about 100
  // independent loads) are issued before the normalisation constants are
  // staged, so the two global round trips overlap.
  float2 *xn = reinterpret_cast<float2 *>(lds + XNORM_OFF);
  const int fcol = tid & (FT - 1), part = tid >> 7;
  int c = -1;
  {
    const int r = r0 + fcol;
    if (r < nrows) c = rows_mode ? (a.list ? a.list[r] : r) : a.c0 + r;
    if (c >= nx * a.g.ny) c = -1;                    // not a column: zero row
  }
  const int kb = part * kPartLev, ke = min(kNZ, kb + kPartLev);
  // slot n holds level kb - 1 + n (slot 0: the level below, none for part 0)
  float th[kPartLev + 1], qq[kPartLev + 1], ul[kPartLev + 1], uh[kPartLev + 1], vl[kPartLev + 1],
      vh[kPartLev + 1];
  float srf[4] = {0.f, 0.f, 0.f, 0.f};
  if (c >= 0) {
    const int i = c % nx, j = c / nx;
    const unsigned g0 = a.g.origin + unsigned(i) + unsigned(j) * a.g.sj;
    const unsigned sk = a.g.sk, sj = a.g.sj;
#pragma unroll
    for (int n = 0; n <= kPartLev; ++n) {
      const int k = kb - 1 + n;
      if (k >= 0 && k < ke) {
        const unsigned g = g0 + unsigned(k) * sk;
        th[n] = ldg(a.th, g);
        qq[n] = ldg(a.q, g);
        ul[n] = ldg(a.u, g - 1);
        uh[n] = ldg(a.u, g);
        vl[n] = ldg(a.v, g - sj);
        vh[n] = ldg(a.v, g);
      }
    }
    if (part == 3) {
      srf[0] = ldg(a.th_s, unsigned(c));
      srf[1] = ldg(a.q_s, unsigned(c));
      srf[2] = ldg(a.f0, unsigned(c));
      srf[3] = ldg(a.ch, unsigned(c));
    }
  }
  for (int f = tid; f < MLP_KIN; f += FTHREADS) xn[f] = make_float2(a.xmean[f], a.xinvstd[f]);
  for (int n = tid; n < MLP_NHID; n += FTHREADS) {
    s_bias[n] = a.b1[n];
    s_bias[MLP_NHID + n] = a.b2[n];
  }
  if (tid < MLP_NOUTP) s_bias[2 * MLP_NHID + tid] = a.b3[tid];
  __syncthreads();
  {
    uint16_t *xr = X + fcol * XLD;
    // normalised BF16 pair (f, f + 1), f even: one 4-byte LDS store
    auto put2 = [&](int f, float x0, float x1) {
      const float2 m0 = xn[f], m1 = xn[f + 1];
      *reinterpret_cast<uint32_t *>(xr + f) = f2bf2((x0 - m0.x) * m0.y, (x1 - m1.x) * m1.y);
    };
    if (c < 0) {
      for (int f = 2 * part; f < MLP_KIN; f += 8) *reinterpret_cast<uint32_t *>(xr + f) = 0u;
    } else {
      LevelVals prev{};
      float fe[5];
#pragma unroll
      for (int n = 0; n <= kPartLev; ++n) {
        const int k = kb - 1 + n;
        if (k >= ke) break;
        if (k < 0) continue;
        LevelVals cur;
        cur.th = float(double(th[n]) + a.theta_off - kThetaRef);
        cur.q = qq[n];
        cur.u = (ul[n] + uh[n]) * 0.5f;
        cur.v = (vl[n] + vh[n]) * 0.5f;
        if (n >= 1) {
          float fv[5];
          level_features(k, cur, prev, fv);
          if (n & 1) {
#pragma unroll
            for (int q5 = 0; q5 < 5; ++q5) fe[q5] = fv[q5];
          } else {
#pragma unroll
            for (int q5 = 0; q5 < 5; ++q5) put2(q5 * kNZ + k - 1, fe[q5], fv[q5]);
          }
        }
        prev = cur;
      }
      if (part == 3) {
        put2(5 * kNZ, float(double(srf[0]) + a.theta_off - kThetaRef), srf[1]);
        put2(5 * kNZ + 2, srf[2], srf[3]);
        for (int f = 5 * kNZ + 4; f < MLP_KIN; f += 2) *reinterpret_cast<uint32_t *>(xr + f) = 0u;
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
  tile_gemm<2, 4, MLP_KIN>(acc, X, XLD, 0, a.w1, n0, lane);
  __syncthreads();   // every wave has read X
  store_hidden<2, 4>(acc, s_bias, n0, H, lane);
  __syncthreads();

  // ---- hidden layer 2: H = relu(H W2^T + b2) ---------------------------------
#pragma unroll
  for (int y = 0; y < 2; ++y)
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[y][x][r] = 0.f;
  tile_gemm<2, 4, MLP_NHID>(acc, H, HLD, 0, a.w2, n0, lane);
  __syncthreads();
  store_hidden<2, 4>(acc, s_bias + MLP_NHID, n0, H, lane);
  __syncthreads();

  // ---- output layer: Y = H W3^T + b3 (normalised tendencies) -----------------
  // wave w: outputs [32 (w % 4), +32) of samples [64 (w / 4), +64)
  f32x16 acc3[1][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc3[0][x][r] = 0.f;
  const int o3 = 32 * (wave & 3), s3 = 64 * (wave >> 2);
  tile_gemm<1, 2, MLP_NHID>(acc3, H, HLD, s3, a.w3, o3, lane);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int o = o3 + 8 * q + 4 * (lane >> 5);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int c = 0; c < 4; ++c) Y[(s3 + 32 * x + (lane & 31)) * YLD + o + c] = acc3[0][x][4 * q + c] + s_bias[2 * MLP_NHID + o + c];
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
  const int col = fcol;
  if (r0 + col >= nrows) return;
  const int cu = a.c0 + r0 + col;
  if (a.judged && judge_sampled(a.seed, a.t, unsigned(cu), a.rate)) return;
  const int ny = a.g.ny;
  const int i = cu % nx, j = cu / nx;
  const unsigned g0 = a.g.origin + unsigned(i) + unsigned(j) * a.g.sj;
  const int di = i < 2 ? nx : (i >= nx - 2 ? -nx : 0);
  const int dj = j < 2 ? ny * int(a.g.sj) : (j >= ny - 2 ? -ny * int(a.g.sj) : 0);
  float *fld = part < 2 ? a.th : a.q;
  const int kbu = (part & 1) ? kHalf : 0;
  const int nk = (part & 1) ? kNZ - kHalf : kHalf;
  const int ob = (part < 2 ? 0 : kNZ) + kbu;
  const float *yr = Y + col * YLD + ob;
  if (a.tend_t) {
    // tendency mode: d(theta)/dt or d(q)/dt at (i, j, k), i fastest
    float *tf = part < 2 ? a.tend_t : a.tend_q;
    for (int k = 0; k < nk; ++k) {
      const float2 ms = yn[ob + k];
      stg(tf, unsigned((kbu + k) * ny + j) * unsigned(nx) + unsigned(i), fmaf(yr[k], ms.y, ms.x));
    }
    return;
  }
  const unsigned gb = g0 + unsigned(kbu) * a.g.sk;
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
