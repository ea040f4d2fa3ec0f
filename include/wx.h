/*
 * wx.h -- C ABI of the structured-grid weather step on one MI355X (gfx950).
 *
 * One step advances density rho and the mixing ratios theta, q on a periodic
 * i/j grid with nz levels: a third-order Runge-Kutta long step of a
 * finite-volume C-grid transport (the dynamical core; paper section "The
 * ASUCA Weather Prediction Model") followed by column-local physics run after
 * the dycore with no horizontal interaction (section "Architecture-Dependant
 * Parallelization Granularity"): implicit vertical diffusion solved by the
 * Thomas algorithm and a radiative-transmissivity k-scan.  The concrete
 * equations are this library's readings; the paper prints none.
 *
 * Storage (section "Architecture-Dependent Storage Order": on GPUs the first
 * parallel index is stride-1; the reduced application dimensions its fields
 * with a horizontal halo only):
 *   - every 3D cell field is i-fastest, then j, then k, with a halo of
 *     WX_HALO cells on each side in i and j and none in k;
 *   - element (i, j, k), i in [-2, nx+2), j in [-2, ny+2), k in [0, nz), lives
 *     at  origin + i + j*stride_j + k*stride_k  (units: elements of the dtype);
 *   - u is the wind on the east face of cell (i,j), v on the north face, both
 *     stored like a cell field; w has nz+1 face levels (k = 0 ground ... nz
 *     lid) with the same i/j layout; w at k = 0 and k = nz is ignored (no flux);
 *   - 2D surface fields (theta_s, q_s, f0, ch) are nx*ny, i fastest, no halo;
 *   - tendency outputs are nx*ny*nz, i fastest, no halo.
 *
 * Ownership: every device buffer is allocated by the caller and only borrowed
 * by the library, which allocates no device memory.  The library owns the
 * wx_state struct and its host-side copies.  All pointers are device pointers
 * unless stated otherwise and must be 16-byte aligned.
 *
 * Errors: every int-returning call returns a wx_status.  Argument and state
 * errors are detected synchronously on the host and leave the device
 * untouched; wx_last_error() then gives a message (per host thread).  Numeric
 * faults on the device (non-finite values, rho <= 0) do not fail a call: they
 * are counted in flags_out, which the caller reads after synchronizing.
 *
 * Concurrency: one host thread per state.  Calls are asynchronous on the given
 * HIP stream and never synchronize the host.  Results are bitwise
 * reproducible for identical inputs, binary and GPU (no floating-point
 * atomics; every reduction has a fixed order).
 */
#ifndef WX_H
#define WX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WX_HALO 2

typedef enum wx_status {
  WX_OK = 0,
  WX_E_INVAL = -1,        /* bad argument (size, pointer, alignment, enum)      */
  WX_E_HIP = -2,          /* a HIP runtime call failed (message has the code)   */
  WX_E_STATE = -3,        /* state incomplete (a required pointer is NULL)      */
  WX_E_UNSUPPORTED = -4   /* valid request this build does not implement        */
} wx_status;

typedef enum wx_dtype { WX_F32 = 0, WX_F64 = 1 } wx_dtype;

typedef enum wx_phys_mode {
  WX_PHYS_OFF = 0,        /* dycore only                                        */
  WX_PHYS_PLAIN = 1,      /* dycore, then implicit diffusion + radiation        */
  WX_PHYS_SURROGATE = 2,  /* dycore, then the learned surrogate on every column */
  WX_PHYS_JUDGED = 3,     /* dycore, surrogate, plain physics on sampled columns
                             as judge, whole-step fallback to the plain physics  */
  WX_PHYS_DATASET = 4     /* wx_physics only: raw feature rows and plain-physics
                             tendency labels of every column (as wx_dataset)    */
} wx_phys_mode;

/* Tunable constants (readings of the paper; defaults in brackets). */
typedef enum wx_param {
  WX_PARAM_GAMMA4 = 0,       /* biharmonic strength, K4 = gamma4 dx^4/dt [2^-8]  */
  WX_PARAM_KMIN = 1,         /* background vertical diffusivity, m^2/s [0.1]     */
  WX_PARAM_MIXLEN = 2,       /* mixing length l, m [50]                          */
  WX_PARAM_KAPPA_Q = 3,      /* absorber extinction, m^2/kg [0.02]               */
  WX_PARAM_CP = 4,           /* heat capacity, J/(kg K) [1004]                   */
  WX_PARAM_TDD = 5,          /* dominance ratio above which the Thomas forward
                                elimination runs in FP64 [64]                    */
  WX_PARAM_THETA_OFFSET = 6, /* theta is stored as theta - offset; used only by
                                the mass sums, which report rho*theta with the
                                offset added back in FP64 [0]                    */
  WX_PARAM_MASS_EVERY = 7,   /* wx_step computes the mass sums on every step
                                whose 1-based index is a multiple of this, and
                                always on the last step; 0 = never [1]          */
  WX_PARAM_JUDGE_SEED = 8,   /* judge sample seed, integer < 2^32 [0]           */
  WX_PARAM_JUDGE_REL = 9,    /* fallback when a pooled RMSE > rel * sigma [0.05] */
  WX_PARAM_JUDGE_RATE = 10,  /* one column in `rate` is sampled, integer 1..2^32-1;
                                fixed once the surrogate workspace is sized [100] */
  WX_PARAM_STEP = 11,        /* index t of the next step (sample hash), integer
                                >= 0; wx_step advances it by nsteps [0]          */
  WX_PARAM_PHYS_KERNEL = 12, /* kernel of the FP32 plain physics: 0 thread per
                                column, column kept in registers (one wave per
                                SIMD; nz 16 and 58); 1 the same, column read
                                again on the way down (two waves per SIMD);
                                2 wave per column, the k-recurrences
                                (elimination, back substitution, optical
                                depth) as scans over the lanes (nz <= 64; same
                                arithmetic in another order: equal within
                                rounding); 3 as 0, each level fetched with two
                                16-byte loads per lane through LDS (field
                                pointers 16-byte aligned); 0, 1 and 3 give the
                                same bits; 4 two lanes per column, the
                                elimination run from the ground and from the
                                lid and joined at mid-column (two waves per
                                SIMD; nz 16 and 58; equal to 0 within
                                rounding; at nz 58 also the judge's sampled
                                columns, bit for bit the whole-grid result) [4] */
  WX_PARAM_STAGE_TILE = 13,  /* tile of the RK3 stage kernel (columns x rows), same
                                results bit for bit: 0 64x8 (stage 2 on 64x12),
                                1 64x4, 2 64x12,
                                3 32x16, 4 128x4, 5 64x8 with each face value,
                                mass flux and Laplacian formed once per tile
                                in LDS instead of once per adjacent cell [0]     */
  WX_PARAM_COUNT = 14
} wx_param;

/* Flags written by wx_step / wx_mass into flags_out[WX_NFLAGS] (cleared at the
 * start of each wx_step call, then accumulated over its steps). */
#define WX_FLAG_NONFINITE 0   /* cells with a non-finite rho, theta or q        */
#define WX_FLAG_RHO_LE0 1     /* cells with rho <= 0                             */
#define WX_FLAG_FP64_COLS 2   /* column solves that took the FP64 elimination    */
#define WX_FLAG_FALLBACK 3    /* judged steps that fell back to the plain physics */
#define WX_NFLAGS 4

typedef struct wx_state {
  /* ---- set by wx_create; read-only for the caller ---- */
  int32_t nx, ny, nz, halo;
  int64_t stride_j;        /* elements between j and j+1                          */
  int64_t stride_k;        /* elements between k and k+1                          */
  int64_t origin;          /* element offset of interior cell (0,0,0)             */
  int64_t field_elems;     /* elements of one 3D cell field (nz planes)           */
  int64_t wfield_elems;    /* elements of w (nz+1 planes)                         */
  double dt, dx;           /* time step [s]; horizontal spacing [m], dy == dx     */
  /* ---- set by the caller before wx_step / wx_physics / wx_mass ---- */
  int32_t dtype;           /* wx_dtype of every field buffer [WX_F32]             */
  int32_t phys_mode;       /* wx_phys_mode used by wx_step [WX_PHYS_PLAIN]        */
  void *stream;            /* hipStream_t used by wx_physics / wx_mass [0]        */
  void *rho, *theta, *q;   /* prognostic fields, field_elems each, updated in place */
  void *u, *v;             /* frozen face winds, field_elems each                 */
  void *w;                 /* frozen vertical wind, wfield_elems                  */
  void *theta_s, *q_s;     /* surface values of theta and q, nx*ny                */
  void *f0;                /* downward flux at the lid [W/m^2], nx*ny             */
  void *ch;                /* surface exchange velocity [m/s], nx*ny              */
  void *workspace;         /* >= wx_workspace_bytes(...) device bytes             */
  double *mass_out;        /* 6 doubles: (sum, compensation) of rho V,
                              rho theta V, rho q V with V = dx dy dz_k            */
  int32_t *flags_out;      /* WX_NFLAGS ints                                      */
  /* surrogate modes only (WX_PHYS_SURROGATE / WX_PHYS_JUDGED; FP32 state, nz 58): */
  void *mlp;               /* trained parameter blob (wx_mlp_bytes)               */
  void *surrogate_work;    /* >= wx_surrogate_work_bytes(...) device bytes        */
  double *judge_out;       /* 6 doubles, last judged step: RMSE theta [K/s], RMSE
                              q [1/s], fallback (0/1), sampled columns, and the
                              fractions of sampled columns whose own RMSE over
                              the levels exceeds the bound (theta, q)            */
  void *impl;              /* private                                             */
} wx_state;

typedef struct wx_tend {
  void *dtheta;            /* nx*ny*nz of the state's dtype: d(theta)/dt [K/s]    */
  void *dq;                /* nx*ny*nz: d(q)/dt [1/s]                             */
  void *features;          /* WX_PHYS_DATASET: [nx*ny][320] FP32 raw feature rows */
  float *labels;           /* WX_PHYS_DATASET: [nx*ny][128] FP32 tendency labels  */
} wx_tend;

/* Create a state for an nx x ny x nz grid (nx, ny >= 4, 3 <= nz <= 1024),
 * time step dt > 0 [s], spacing dx > 0 [m] and level thicknesses dz[nz] > 0
 * (host array, k = 0 at the ground, copied).  Returns NULL on error. */
wx_state *wx_create(int nx, int ny, int nz, double dt, double dx, const double *dz);

/* Free the state.  The caller must have synchronized every stream it used. */
void wx_destroy(wx_state *s);

/* Message for the last non-OK return on this host thread ("" if none). */
const char *wx_last_error(void);

/* Device workspace bytes wx_step / wx_physics / wx_mass need for this dtype:
 * two RK stage copies of (rho, theta, q), the FP64 column-elimination scratch,
 * block partials of the mass sums and a few constants. */
size_t wx_workspace_bytes(const wx_state *s, int dtype);

/* Device workspace of the surrogate modes: the judge's sample list, the
 * plain tendencies and network outputs of the sampled columns, the judge's
 * block partials and counters; sized for the current WX_PARAM_JUDGE_RATE. */
size_t wx_surrogate_work_bytes(const wx_state *s);

/* Set / get a wx_param.  Values must be finite; GAMMA4, KMIN, MIXLEN, KAPPA_Q
 * >= 0, CP > 0, TDD >= 0, MASS_EVERY >= 0 (integral). */
int wx_set_param(wx_state *s, int param, double value);
int wx_get_param(const wx_state *s, int param, double *value);

/* Fill the periodic halo ring (corners included) of rho, theta, q, u and v
 * from the interior, asynchronously on `stream`. */
int wx_halo(wx_state *s, void *stream);

/* Advance the state by nsteps >= 0 steps on `stream` (also stored as
 * s->stream).  Per call: halo fill, then per step three RK stages (the long
 * step of section "The ASUCA Weather Prediction Model") and the physics of
 * phys_mode: none, the plain column physics, the surrogate on every column,
 * or the judged surrogate (see the surrogate section below).  Fields are updated in place; the halo
 * ring is kept current.  Mass sums of the final state go to mass_out (see
 * WX_PARAM_MASS_EVERY); flags_out is cleared and then accumulated. */
int wx_step(wx_state *s, int nsteps, void *stream);

/* Physics tendencies of the current state on s->stream, state unchanged.
 * Requires a current halo on u and v (wx_halo or wx_step).
 *   WX_PHYS_PLAIN: t->dtheta = delta_theta/dt + H, t->dq = delta_q/dt of one
 *     implicit-diffusion + radiation step of length dt (any dtype, any nz);
 *   WX_PHYS_SURROGATE: the learned surrogate's tendencies of every column
 *     (FP32 state, nz 58, s->mlp and s->surrogate_work set);
 *   WX_PHYS_JUDGED: the surrogate's tendencies judged on the columns sampled
 *     for step index WX_PARAM_STEP (not advanced): sampled columns carry the
 *     plain tendencies, and every column does when the pooled RMSE exceeds
 *     the bound (s->judge_out receives the verdict, as in wx_step);
 *   WX_PHYS_DATASET: t->features and t->labels as wx_dataset fills them
 *     (t->dtheta / t->dq unused). */
int wx_physics(wx_state *s, wx_tend *t, int mode);

/* Compensated FP64 mass sums of the current state into mass_out (6 doubles),
 * on s->stream; fixed reduction order, so bitwise reproducible. */
int wx_mass(wx_state *s);

/* Largest ceil(nx/64)*ny that wx_mass_noalloc accepts (its block partials
 * live in a fixed device array of 6 doubles per block). */
#define WX_MASS_NOALLOC_MAX_PARTS 40960

/* wx_mass for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and summation order as wx_mass, so bitwise the same mass_out, but
 * the block partials and level volumes live in a static per-device array of
 * 8 KiB + WX_MASS_NOALLOC_MAX_PARTS * 48 B (1.9 MiB) that the library keeps
 * until the process ends; s->workspace is neither needed nor touched.  Needs
 * rho, theta, q, mass_out and flags_out; grids with ceil(nx/64)*ny above
 * WX_MASS_NOALLOC_MAX_PARTS (and nz above 1024) are rejected with WX_E_INVAL
 * before any device work.  Calls no hipMalloc/hipFree.  Every call on one
 * GPU shares that array: calls that overlap in time on one GPU (two streams,
 * two host threads) race and must be serialized by the caller.  Runs on
 * s->stream; adds fault counts to flags_out like wx_mass. */
int wx_mass_noalloc(wx_state *s);

/* Timing instrument: run nsteps steps like wx_step with a HIP event around
 * every kernel launch (same stream), synchronize, and write the average
 * duration in ms of each launch class to ms_out[0..n_out): 0 halo fill,
 * 1 stage 1, 2 stage 2, 3 stage 3, 4 physics (mass partials when the plain
 * physics is off), 5 mass finalisation; with the surrogate: 6 judge prelude
 * (sampling, plain physics and inference of the sampled columns, verdict),
 * 7 the fused surrogate over all columns, 8 sampled-column apply plus the
 * fallback physics launch.  Classes that did not run read 0.  The events
 * themselves add small gaps between launches. */
int wx_profile_step(wx_state *s, int nsteps, void *stream, double *ms_out, int n_out);

/* Plain device copy kernel of `bytes` (multiple of 16) from src to dst on
 * `stream`: the reference for bandwidth and for scaling HBM counters. */
int wx_copy_probe(void *dst, const void *src, size_t bytes, void *stream);

/* ======================================================================
 * Learned surrogate of the column physics (BF16 matrix-core MLP).
 *
 * A 294-512-512-116 ReLU network maps a column's physics inputs to its
 * theta and q tendencies.  GEMM operands are BF16 (round to nearest even),
 * accumulation FP32; weights are kept FP32 with BF16 copies.  Layouts:
 *   features  [n][WX_MLP_KIN] : five profiles over k = 0..57 from theta' =
 *             theta - 300 K, q and the cell-centred winds (u, v): theta'_0
 *             then theta'_k - theta'_{k-1}; q_0 then q_k - q_{k-1}; |(u,v)_0|
 *             then the shear S_k = |(u,v)_k - (u,v)_{k-1}|; 0 then S_k times
 *             the theta' difference; 0 then S_k times the q difference; then
 *             theta_s - 300 K, q_s, F0, C_h; zero padding; column c = i + nx j;
 *   targets   [n][WX_MLP_NOUTP]: 58 theta tendencies [K/s], 58 q tendencies
 *             [1/s], zero padding.
 * All buffers are device memory owned by the caller.  The parameter blob is
 * one buffer of wx_mlp_bytes() bytes whose sections start at
 * wx_mlp_offset(section); the caller may read or write any section (FP32
 * weights written by the caller take effect after wx_mlp_refresh).
 * ====================================================================== */
#define WX_MLP_NZ 58
#define WX_MLP_NIN 294
#define WX_MLP_KIN 320
#define WX_MLP_NHID 512
#define WX_MLP_NOUT 116
#define WX_MLP_NOUTP 128

typedef enum wx_mlp_section {
  /* FP32 parameters: W1 [512][320], b1 [512], W2 [512][512], b2 [512],
     W3 [128][512], b3 [128] (padding entries stay zero) */
  WX_MLP_W1 = 0, WX_MLP_B1 = 1, WX_MLP_W2 = 2, WX_MLP_B2 = 3, WX_MLP_W3 = 4, WX_MLP_B3 = 5,
  WX_MLP_GRAD = 6,     /* + 0..5: gradients of the last wx_mlp_forward_backward, same shapes */
  WX_MLP_ADAM_M = 12,  /* + 0..5: Adam first moments */
  WX_MLP_ADAM_V = 18,  /* + 0..5: Adam second moments */
  WX_MLP_W1_BF16 = 24, WX_MLP_W2_BF16 = 25, WX_MLP_W3_BF16 = 26,  /* BF16 copies, same shapes */
  WX_MLP_W2T_BF16 = 27,  /* W2 transposed [512][512] */
  WX_MLP_W3T_BF16 = 28,  /* W3 transposed [512][128] */
  WX_MLP_X_MEAN = 29, WX_MLP_X_INVSTD = 30,  /* FP32 [320]: feature mean and 1/std (0 on padding) */
  WX_MLP_Y_MEAN = 31, WX_MLP_Y_STD = 32,     /* FP32 [128]: target mean and scale (1 on padding) */
  WX_MLP_SIGMA = 33,    /* FP32 [2]: pooled std of the theta and q tendencies */
  WX_MLP_SIGMA64 = 34,  /* FP64 [2]: the same in FP64 */
  /* W1, W2, W3 in BF16 again, one after the other, each in matrix-core
     fragment order: the 32-row x 16-k block (R, S) of a [N][K] matrix is 512
     contiguous values, lane l holding row 32R + l%32 at k = 16S + 8(l/32)
     .. +7, so a wavefront reads each block as one 1 KiB run (the operand
     layout of the fused surrogate kernel; written with the BF16 copies) */
  WX_MLP_WPACK_BF16 = 35,
  WX_MLP_NSECTIONS = 36
} wx_mlp_section;

size_t wx_mlp_bytes(void);
/* Byte offset of a section in the blob; -1 for an unknown section. */
int64_t wx_mlp_offset(int section);
/* He-uniform weights (+-sqrt(6/fan_in), element e of tensor t drawn from
 * SplitMix64((seed << 32) | (t << 28) | e)), zero biases, gradients and
 * moments, identity normalisation, BF16 copies. */
int wx_mlp_init(void *blob, uint64_t seed, void *stream);
/* Rebuild the BF16 copies from the FP32 weights. */
int wx_mlp_refresh(void *blob, void *stream);

/* Normalisation: FP64 mean and population std per feature over n raw rows
 * (std < 1e-12 is replaced by 1); per target its mean and the pooled std of
 * its variable (theta tendencies or q tendencies, over all rows and levels),
 * which is also stored as sigma; all in the blob.
 * scratch: wx_mlp_norm_scratch_bytes(n). */
size_t wx_mlp_norm_scratch_bytes(size_t n);
int wx_mlp_fit_norm(void *blob, const float *x_raw, const float *y_raw, size_t n, void *scratch, void *stream);
/* x_out [n][320] BF16 = (x - mean) / std; y_out [n][128] FP32 (y may be NULL). */
int wx_mlp_normalize(const void *blob, const float *x_raw, const float *y_raw, size_t n, void *x_out,
                     float *y_out, void *stream);

/* Training on normalised data x [N][320] BF16 and y [N][128] FP32: the batch
 * is rows[0..batch) (device int32).  forward_backward writes the gradients of
 * mean((y_hat - y)^2) over the batch and the 116 outputs into the GRAD
 * sections and the sum of squared errors into loss_sum[0] (device).  adam
 * applies one Adam step (t >= 1, beta 0.9 / 0.999, eps 1e-8) and refreshes
 * the BF16 copies.  work: wx_mlp_work_bytes(batch).  batch is 1..65536. */
size_t wx_mlp_work_bytes(int batch);
int wx_mlp_forward_backward(void *blob, void *work, const void *x, const float *y, const int32_t *rows,
                            int batch, float *loss_sum, void *stream);
int wx_mlp_adam(void *blob, float lr, int t, void *stream);
int wx_mlp_train_step(void *blob, void *work, const void *x, const float *y, const int32_t *rows, int batch,
                      float lr, int t, float *loss_sum, void *stream);

/* The row order of a training epoch, drawn on the device: out[i] = P(i) for
 * i < m, where P is a permutation of 0..n-1 fixed by (seed, epoch): a
 * four-round Feistel network on the smallest even bit width holding n, whose
 * round function is SplitMix64 of (seed, epoch, round, half), walked until it
 * lands below n.  Deterministic, one independent evaluation per element.
 * out: device int32[m], 0 <= m <= n <= 2^30; WX_E_INVAL otherwise. */
int wx_mlp_shuffle(uint64_t seed, uint64_t epoch, int n, int m, int32_t *out, void *stream);

/* Inference: y_out [n][128] FP32 normalised outputs for x [n][320] BF16.
 * work: wx_mlp_infer_work_bytes(n). */
size_t wx_mlp_infer_work_bytes(int n);
int wx_mlp_infer(const void *blob, void *work, const void *x, int n, float *y_out, void *stream);

/* Fused surrogate inference on columns of the current FP32 state (nz = 58)
 * on s->stream: row r < n is column cols[r] (device int32; an index outside
 * 0..nx*ny-1 gives the row of zero features) or column r when cols is NULL
 * (then n <= nx*ny).  rows_out [n][WX_MLP_NOUTP] (device FP32) receives the
 * normalised network outputs; the tendencies are rows_out * y_std + y_mean.
 * The kernel builds the feature rows from the state and the blob's
 * statistics and runs the three layers without leaving the chip; the outputs
 * equal wx_features(normalized = 1) followed by wx_mlp_infer bit for bit.
 * This is the kernel that the surrogate step modes run over every column. */
int wx_surrogate_rows(wx_state *s, const void *blob, const int32_t *cols, int n, float *rows_out);

/* Feature rows of the current state on s->stream (nz must be 58): raw FP32
 * (normalized = 0, blob unused) or normalised BF16 with the blob's statistics.
 * out holds nx*ny rows of WX_MLP_KIN values. */
int wx_features(wx_state *s, int normalized, void *out, const void *blob);
/* Training data of the current state on s->stream (FP32 state, nz = 58): raw
 * feature rows and the plain-physics tendency rows (targets), nx*ny each. */
int wx_dataset(wx_state *s, float *x_raw, float *y_raw);

/* ---- The paper's reduced weather application ---------------------------
 * Section "Reduced Weather Application" and its appendix sources (diffusion,
 * physical processes, radiation, heat exchange, time integration).  One FP64
 * field E over i = 0..nx+1, j = 0..ny+1 (a one-cell ring around the nx x ny
 * interior) and nz levels, stored dense with i fastest, then j, then k:
 * element (i, j, k) at k (nx+2)(ny+2) + j (nx+2) + i, k = 0 the bottom.
 * surf and pbl are [ny+2][nx+2] FP64 (the surface and boundary-layer values
 * of each column).  All pointers are device memory, 8-byte aligned; the
 * caller owns them.
 *
 * A step is the printed one: on every column radiation adds 0.1 to each
 * level, then the bottom level loses 0.01 (E - surf) and the top level
 * 0.01 (E - pbl); then one explicit-Euler diffusion step with diffusion
 * number nu writes the other array: interior columns take the 7-point rule
 * E (1 - 6 nu) + nu (six neighbours) inside and the 6-point rule
 * E (1 - 5 nu) + nu (five neighbours) on the bottom and top levels; ring
 * rows and then ring columns (corners included) take
 * E (1 - 2 nu) + nu (inner neighbour + opposite ring cell).  Sums run in the
 * printed order and no multiply-add is fused: results equal the printed
 * FP64 program bit for bit.
 *
 * Requires nx, ny >= 1, nz >= 2, (nx+2)(ny+2) nz <= 2^29 and a finite nu;
 * otherwise WX_E_INVAL and nothing is launched. */

/* One step from e_in into e_out (distinct arrays) on stream. */
int wx_rw_step(const double *e_in, double *e_out, const double *surf, const double *pbl, int nx, int ny, int nz,
               double nu, void *stream);
/* nsteps steps alternating between e0 and e1 (the printed pointer swap),
 * starting from e0; *which (host) receives 0 or 1, the array that holds the
 * result (0 when nsteps = 0). */
int wx_rw_run(double *e0, double *e1, const double *surf, const double *pbl, int nx, int ny, int nz, double nu,
              int nsteps, int *which, void *stream);
/* wx_rw_run with a chosen thread-block shape block_x x block_y (the paper's
 * table "Block Size Impact on Execution Time" compares its compiler's
 * default 128 x 1 with 32 x 16): one of 64x8 (wx_rw_run's), 32x16, 128x1,
 * 64x4, 128x4, else WX_E_UNSUPPORTED.  Every shape does the same arithmetic
 * per cell, so results equal wx_rw_run's bit for bit.  Same arguments,
 * requirements and errors as wx_rw_run otherwise. */
int wx_rw_run_block(double *e0, double *e1, const double *surf, const double *pbl, int nx, int ny, int nz, double nu,
                    int nsteps, int *which, int block_x, int block_y, void *stream);
/* The same steps on the KIJ storage order (section "Performance Portable
 * Storage Order": k fastest, then i, then j; element (i, j, k) at
 * (j (nx+2) + i) nz + k), with one thread per column marching k, the direct
 * GPU mapping of that order.  Results equal wx_rw_run's bit for bit (after
 * the reordering); it exists to measure what the order costs on this GPU.
 * Same arguments, requirements and errors as wx_rw_run. */
int wx_rw_run_kij(double *e0, double *e1, const double *surf, const double *pbl, int nx, int ny, int nz, double nu,
                  int nsteps, int *which, void *stream);

/* ======================================================================
 * Fast modes: HEVI short steps of the linear acoustic-gravity system.
 *
 * Section "The ASUCA Weather Prediction Model" splits sound and gravity
 * waves from the Runge-Kutta long step: they advance in shorter steps of a
 * second-order Runge-Kutta scheme, horizontally explicit and vertically
 * implicit (HEVI); section "Hybrid ASUCA Strong Scaling GPU Results" names
 * them as the costliest module.  The paper prints no equations; this library
 * reads them as the linearised system about a resting state with kinematic
 * pressure pi and buoyancy b,
 *   du/dt = -dpi/dx, dv/dt = -dpi/dy, dw/dt = -dpi/dz + b, db/dt = -N^2 w,
 *   dpi/dt = -c^2 (du/dx + dv/dy + dw/dz),
 * on the dycore's C-grid (u on east faces, v on north faces, pi at cell
 * centres, w and b on the nz + 1 level faces with w = b = 0 at the ground
 * and lid; vertical differences over dz_k at cells and (dz_{k-1} + dz_k)/2 at
 * faces).  A short step of length tau is two stages from its start X, with
 * h = tau/2 and then h = tau, each taking the previous stage's pi in the
 * horizontal and treating the vertical terms with the trapezoidal rule:
 *   u' = u - h dpi_prev/dx,  v' = v - h dpi_prev/dy,  D = du'/dx + dv'/dy,
 *   (1 + h^2 N^2/4) wm - (h^2 c^2/4) d/dz(dwm/dz)
 *        = w + (h/2)(-dpi/dz + b) + (h^2 c^2/4) dD/dz   (a tridiagonal solve
 *          per column over the interior faces),
 *   w' = 2 wm - w,  b' = b - h N^2 wm,  pi' = pi - h c^2 (D + dwm/dz).
 *
 * Layout: cell fields (u, v, pi) exactly like wx_state's cell fields (i
 * fastest, 2-cell halo in i and j, stride_j = roundup(nx + 4, 64)); face
 * fields (w, b) have nz + 1 planes of the same shape.  All device buffers
 * belong to the caller.
 * ====================================================================== */

typedef struct wx_hevi_grid {
  int32_t nx, ny, nz, dtype;     /* nx, ny >= 4, 2 <= nz <= 1024; WX_F32 / WX_F64     */
  int64_t stride_j, stride_k;    /* elements, as for wx_state                       */
  int64_t origin;                /* element offset of interior (0,0,0)              */
  int64_t cell_elems;            /* elements of one cell field (nz planes)          */
  int64_t face_elems;            /* elements of one face field (nz + 1 planes)      */
  double dx;                     /* horizontal spacing [m], dy == dx                */
  double tau;                    /* short step [s]                                  */
  double c_sound, n_bv;          /* sound speed [m/s] > 0, buoyancy frequency [1/s] */
  int32_t kernel;                /* 2 (set by init): for nz 16 and 58 two lanes per
                                    column, the vertical system eliminated from the
                                    ground and from the lid and joined at face
                                    nz/2; 0: for nz 16 and 58 one lane per column,
                                    the column's intermediates in registers; 1:
                                    park them in the outputs (any nz; also what 0
                                    and 2 do for other nz); all give the same
                                    results within rounding                       */
  int32_t pad;
} wx_hevi_grid;

/* Fill *g for the given grid and constants (host only).  WX_E_INVAL on bad
 * sizes or non-finite / non-positive dx, tau, c (N >= 0). */
int wx_hevi_grid_init(wx_hevi_grid *g, int nx, int ny, int nz, int dtype, double dx, double tau, double c_sound,
                      double n_bv);

/* Device workspace wx_hevi_run needs: the two stages' coefficient tables,
 * the first stage's pi and parked right-hand side, and a second copy of the
 * five fields for the ping-pong between steps.  0 for a bad grid. */
size_t wx_hevi_workspace_bytes(const wx_hevi_grid *g);

/* Advance (u, v, w, b, pi) by nsteps >= 0 short steps of length g->tau on
 * `stream`, in place (after the last step the fields are in the caller's
 * buffers; the halo rings of u, v and pi are filled at entry and kept
 * current).  dz: host array of nz level thicknesses > 0 (k = 0 at the
 * ground).  Two kernel launches per step (the first stage writes only its
 * pi).  The call uploads the small coefficient tables from host memory and
 * synchronizes `stream` once for that upload, before any launch; the steps
 * themselves are asynchronous.  WX_E_INVAL on NULL or
 * misaligned pointers, bad dz or nsteps < 0, before any device work. */
int wx_hevi_run(const wx_hevi_grid *g, const double *dz, void *u, void *v, void *w, void *b, void *pi,
                void *workspace, int nsteps, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* WX_H */
