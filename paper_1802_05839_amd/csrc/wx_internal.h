// Internal launch interface between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wx {

// Geometry shared by every kernel.  Element offsets fit in 32 bits (checked
// when the state is created), so kernels index with 32-bit offsets from a
// uniform base pointer.
struct Geom {
  int nx, ny, nz;
  unsigned sj, sk, origin;  // element strides and offset of interior (0,0,0)
};

// Element access through a 32-bit byte offset from a uniform base pointer, so
// that loads and stores use the scalar-base + 32-bit vector-offset address
// form (every buffer is smaller than 4 GiB; checked when the state is created).
template <typename T>
__device__ __forceinline__ T ldg(const T *base, unsigned idx) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + idx * unsigned(sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void stg(T *base, unsigned idx, T v) {
  *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + idx * unsigned(sizeof(T))) = v;
}
template <typename T>
__device__ __forceinline__ T &ref(T *base, unsigned idx) {
  return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + idx * unsigned(sizeof(T)));
}

// Address of element `d` (a uniform displacement, possibly negative) from p.
// Kernels keep every uniform part of an address (level * stride_k, -1, -sj,
// ...) in the scalar base pointer and only the per-thread part in the 32-bit
// vector offset, so each load is `global_load v, v_off, s[base]` with a
// per-thread offset that never changes inside the k loop.
template <typename T>
__device__ __forceinline__ T *plane(T *p, long long d) {
  return p + d;
}

// Workgroups are dispatched round-robin over the 8 XCDs; map dispatch index b
// of n so that XCD x works on the contiguous logical range [x*q + min(x, r),
// ...), and tiles that share halo rows share one L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = b & 7, slot = b >> 3;
  return x * q + min(x, r) + slot;
}
// The same bands, each walked from its end: a launch that follows one walking
// forward starts on what that launch wrote last, part of which the
// memory-side cache still holds.
__device__ __forceinline__ int xcd_remap_rev(int b, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = b & 7, slot = b >> 3;
  const int len = q + (x < r ? 1 : 0);
  return x * q + min(x, r) + (len - 1 - slot);
}

// Neumaier-compensated FP64 accumulator (sum s, compensation c).
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

// Sum of an int over the 64 lanes of a wave (lane 0 holds the result).
__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Reciprocal in the arithmetic precision: the hardware estimate (1 ulp) in
// FP32, an exact division in FP64.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

template <typename T>
struct StageArgs {
  const T *in_r, *in_t, *in_q;     // stage input (read with its 2-cell halo)
  const T *bs_r, *bs_t, *bs_q;     // step base (read at the cell only)
  T *out_r, *out_t, *out_q;        // stage output (cell + periodic halo images)
  const T *u, *v, *w;              // frozen winds
  const T *rdz;                    // 1/dz_k
  Geom g;
  T h, rdx, k4;                    // stage step, 1/dx, biharmonic coefficient
  int nbx, nblocks;                // tiles in i, total tiles
  int reverse;                     // walk each XCD's band of tiles from its end
};

template <typename T>
struct PhysArgs {
  T *rho, *th, *q;                 // post-dycore state (updated in place in mode 0)
  const T *u, *v;
  const T *th_s, *q_s, *f0, *ch;   // 2D surface fields (nx*ny)
  T *tend_t, *tend_q;              // mode 1 outputs (nx*ny*nz) or null
  const T *dz, *rdzi;              // dz_k; 1/dz_{k+1/2} (nz-1 used)
  const double *vol;               // dx*dy*dz_k
  double *scratch;                 // column elimination scratch [3][nz][nx*ny]
  double *partials;                // mass partials, 6 per block
  int *flags;                      // WX_NFLAGS counters
  Geom g;
  T dt, kmin, l2, kappa, cp, tdd;
  double theta_off;
  int mode;                        // 0: update state, 1: write tendencies
  int do_mass;                     // mode 0: accumulate mass partials
  int use_lds;                     // FP32 elimination stored in LDS
  int tend_rows;                   // mode 1: rows [col][128] (theta 0..nz-1, q nz..2nz-1, zero pad)
  const int *col_list;             // mode 1: columns list[s], s < min(*n_list, list_cap); row s
  const int *n_list;
  int list_cap;
  const int *run_if;               // when set, the launch does nothing unless *run_if != 0
  int variant;                     // FP32 nz 16/58 kernel: PHYS_VARIANT_*
  int reverse;                     // two-lane kernel, whole grid: walk each XCD's band from its end
};

// Variants of the FP32 register-column physics kernel (nz 16 and 58).
constexpr int PHYS_VARIANT_KEEP = 0;     // column kept in registers, one wave per SIMD
constexpr int PHYS_VARIANT_REREAD = 1;   // column read again on the way down, two waves per SIMD
constexpr int PHYS_VARIANT_SCAN = 2;     // one wave per column, the k-recurrences as lane scans (nz <= 64)
constexpr int PHYS_VARIANT_WIDE = 3;     // as KEEP, the upward pass fetching each level with 16-byte loads per lane
constexpr int PHYS_VARIANT_SPLIT = 4;    // two lanes per column: two-sided elimination, two waves per SIMD (nz 16, 58)
constexpr int PHYS_SCAN_COLS = 32;       // columns per block of the scan kernel
inline int phys_scan_blocks(int nx, int ny) { return ((nx + PHYS_SCAN_COLS - 1) / PHYS_SCAN_COLS) * ny; }
hipError_t launch_physics_scan(const PhysArgs<float> &a, hipStream_t s);


template <typename T>
struct MassArgs {
  const T *rho, *th, *q;
  const double *vol;
  double *partials;
  int *flags;
  Geom g;
  double theta_off;
};

// Per-level coefficients of the HEVI vertical solve for one stage length h:
// face f (between cells f-1 and f, f >= 1): spacing dzf and 1/dzf, coupling
// lo = (h^2 c^2 / 4) / (dzf dz_{f-1}), the Thomas factors inv = 1/(diag +
// lo c'_{f-1}) and c' = -hi inv; cell f: dz and 1/dz.
template <typename T>
struct HeviCoef {
  T dzf, rdzf, lo, inv, cp, dz, rdz, pad;
};

template <typename T>
struct HeviArgs {
  const T *u, *v, *w, *b, *pi;     // stage base (the short step's start)
  const T *pp;                     // pi of the previous stage (horizontal gradient)
  T *u_o, *v_o, *w_o, *b_o, *pi_o; // outputs (u, v, w, b only in the second stage)
  T *e_o;                          // face field parking the eliminated right-hand side
  const HeviCoef<T> *coef;         // [nz]
  const HeviCoef<T> *coef2;        // [nz] two-sided factors (kernel 2): see hevi_host
  Geom g;
  T h, h2, a4, hc2, hn2, dx, rdx;  // h, h/2, h^2 c^2/4, h c^2, h N^2, dx, 1/dx
};

// kernel: 0 column in registers (nz 16, 58), 1 parked in the outputs, 2 two
// lanes per column with the two-sided factors (nz 16, 58)
template <typename T>
hipError_t launch_hevi_stage(const HeviArgs<T> &a, bool full, int kernel, hipStream_t s);

constexpr int PHYS_BX = 64;        // columns per physics block (one wave)
constexpr int PHYS_LDS_NZ_MAX = 80;

template <typename T>
hipError_t launch_halo(T *const *fields, int nf, int nplanes, const Geom &g, hipStream_t s);
template <typename T>
hipError_t launch_stage(const StageArgs<T> &a, int stage, int tile, hipStream_t s);
template <typename T>
hipError_t launch_physics(const PhysArgs<T> &a, hipStream_t s);
template <typename T>
hipError_t launch_mass(const MassArgs<T> &a, hipStream_t s);
hipError_t launch_mass_final(const double *partials, int nparts, double *out, hipStream_t s);
hipError_t launch_fill_i32(int *p, int n, int value, hipStream_t s);
constexpr int TEND_ROW = 128;      // row width of the row-major tendency layout
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
hipError_t launch_rw_step(const double *e, double *out, const double *surf, const double *pbl, int nx, int ny,
                          int nz, double nu, bool kij, hipStream_t s, int bx = 64, int by = 8);
bool rw_block_supported(int bx, int by);

// RK3 stage tile shapes (columns in i x rows in j).  0 is the production
// 64 x 8 (one wave per row); 1-4 are the block-shape ablation.
struct StageShape {
  int bx, by;
};
// 5 is the 64 x 8 kernel that forms each face and Laplacian once per tile.
constexpr int STAGE_TILE_VARIANTS = 6;
constexpr int STAGE_TILE_SHARED = 5;
inline StageShape stage_shape(int tile) {
  switch (tile) {
    case 0: return {64, 8};
    case 1: return {64, 4};
    case 2: return {64, 12};
    case 3: return {32, 16};
    case 4: return {128, 4};
    case 5: return {64, 8};
    default: return {0, 0};
  }
}
inline int stage_tiles_x(int nx, int tile) { return (nx + stage_shape(tile).bx - 1) / stage_shape(tile).bx; }
inline int stage_tiles_y(int ny, int tile) { return (ny + stage_shape(tile).by - 1) / stage_shape(tile).by; }
inline int phys_blocks(int nx, int ny) { return ((nx + PHYS_BX - 1) / PHYS_BX) * ny; }
inline int phys_reg_blocks(int nx, int ny) { return ((nx + 63) / 64) * ((ny + 3) / 4); }
// physics kernel variant for a state: register-resident columns for FP32 and these level counts
inline bool phys_uses_reg(int elem_size, int nz) { return elem_size == 4 && (nz == 58 || nz == 16); }
inline bool phys_uses_scan(int elem_size, int nz, int variant) {
  return elem_size == 4 && nz <= 64 && variant == PHYS_VARIANT_SCAN;
}
inline int phys_split_blocks(int nx, int ny) { return ((nx + 31) / 32) * ((ny + 3) / 4); }
// levels of q the split kernel keeps in LDS, and its dynamic LDS (c', rho and
// those q levels per lane; with the static arrays under 80 KB per block)
constexpr int PHYS_SPLIT_QL = 20;
inline size_t phys_split_lds(int nz) {
  const int h = nz / 2;
  return size_t(2 * h + (PHYS_SPLIT_QL < h ? PHYS_SPLIT_QL : h)) * 256 * sizeof(float);
}
inline int phys_partials(int elem_size, int nx, int ny, int nz, int variant = PHYS_VARIANT_KEEP) {
  if (phys_uses_scan(elem_size, nz, variant)) return phys_scan_blocks(nx, ny);
  if (phys_uses_reg(elem_size, nz) && variant == PHYS_VARIANT_SPLIT) return phys_split_blocks(nx, ny);
  return phys_uses_reg(elem_size, nz) ? phys_reg_blocks(nx, ny) : phys_blocks(nx, ny);
}

}  // namespace wx
