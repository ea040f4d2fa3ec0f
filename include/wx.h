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
  WX_PHYS_PLAIN = 1       /* dycore, then implicit diffusion + radiation        */
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
  WX_PARAM_COUNT = 8
} wx_param;

/* Flags written by wx_step / wx_mass into flags_out[WX_NFLAGS] (cleared at the
 * start of each wx_step call, then accumulated over its steps). */
#define WX_FLAG_NONFINITE 0   /* cells with a non-finite rho, theta or q        */
#define WX_FLAG_RHO_LE0 1     /* cells with rho <= 0                             */
#define WX_FLAG_FP64_COLS 2   /* column solves that took the FP64 elimination    */
#define WX_FLAG_RESERVED 3
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
  void *impl;              /* private                                             */
} wx_state;

typedef struct wx_tend {
  void *dtheta;            /* nx*ny*nz of the state's dtype: d(theta)/dt [K/s]    */
  void *dq;                /* nx*ny*nz: d(q)/dt [1/s]                             */
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

/* Set / get a wx_param.  Values must be finite; GAMMA4, KMIN, MIXLEN, KAPPA_Q
 * >= 0, CP > 0, TDD >= 0, MASS_EVERY >= 0 (integral). */
int wx_set_param(wx_state *s, int param, double value);
int wx_get_param(const wx_state *s, int param, double *value);

/* Fill the periodic halo ring (corners included) of rho, theta, q, u and v
 * from the interior, asynchronously on `stream`. */
int wx_halo(wx_state *s, void *stream);

/* Advance the state by nsteps >= 0 steps on `stream` (also stored as
 * s->stream).  Per call: halo fill, then per step three RK stages (the long
 * step of section "The ASUCA Weather Prediction Model") and, if phys_mode is
 * WX_PHYS_PLAIN, the column physics.  Fields are updated in place; the halo
 * ring is kept current.  Mass sums of the final state go to mass_out (see
 * WX_PARAM_MASS_EVERY); flags_out is cleared and then accumulated. */
int wx_step(wx_state *s, int nsteps, void *stream);

/* Physics tendencies of the current state on s->stream, state unchanged.
 * mode must be WX_PHYS_PLAIN: t->dtheta = delta_theta/dt + H, t->dq = delta_q/dt
 * of one implicit-diffusion + radiation step of length dt.  Requires a current
 * halo on u and v (wx_halo or wx_step). */
int wx_physics(wx_state *s, wx_tend *t, int mode);

/* Compensated FP64 mass sums of the current state into mass_out (6 doubles),
 * on s->stream; fixed reduction order, so bitwise reproducible. */
int wx_mass(wx_state *s);

/* Timing instrument: run nsteps steps like wx_step with a HIP event around
 * every kernel launch (same stream), synchronize, and write the average
 * duration in ms of each launch class to ms_out[0..n_out): 0 halo fill,
 * 1 stage 1, 2 stage 2, 3 stage 3, 4 physics, 5 mass finalisation.  The
 * events themselves add small gaps between launches. */
int wx_profile_step(wx_state *s, int nsteps, void *stream, double *ms_out, int n_out);

/* Plain device copy kernel of `bytes` (multiple of 16) from src to dst on
 * `stream`: the reference for bandwidth and for scaling HBM counters. */
int wx_copy_probe(void *dst, const void *src, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* WX_H */
